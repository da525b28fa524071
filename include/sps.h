/*
 * sps.h -- C ABI of the MI355X single-pulse search hot path.
 *
 * The library computes, on one AMD Instinct MI355X (gfx950):
 *   1. brute-force incoherent dedispersion of a channelised 8-bit filterbank
 *      over a grid of trial DMs (ASTROFLOW, arXiv:2511.02328, Sec. 2.3: the
 *      direct method of cost N_DM N_t N_f, with per-channel integer delays
 *      from Eq. (KDM) rounded as in Eq. (coarse_delay));
 *   2. a boxcar matched-filter S/N search over the DM-time plane (Sec. 1,
 *      step (iii) of the standard single-pulse workflow);
 *   3. candidate detection producing DM, arrival time referenced to the top
 *      of the band, width and S/N (Sec. 2, the candidate record).
 *
 * Conventions for every call:
 *   - All functions return sps_status.  No exception, abort or exit crosses
 *     the ABI.  On failure a message is available from sps_last_error()
 *     (thread-local, valid until the next call on the same thread).
 *   - Arguments are validated before any work is enqueued; a call that
 *     returns SPS_ERR_INVALID_ARG / RANGE / OVERFLOW has done nothing.
 *   - "device" pointers are HIP device memory on the device that was current
 *     when the plan was created; "host" pointers are ordinary host memory.
 *     The caller owns every buffer it passes; the library never frees or
 *     retains them after the call returns (device buffers must stay valid
 *     until the enqueued work completes).
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *     sps_dedisperse and sps_boxcar_snr are asynchronous with respect to the
 *     host; sps_detect synchronises the stream before it returns.
 *   - A plan may be used by one stream at a time (it owns scratch memory).
 *   - Errors from kernels that ran earlier on the stream surface as
 *     SPS_ERR_DEVICE from the call that observes them.
 */
#ifndef SPS_H
#define SPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPS_OK = 0,
  SPS_ERR_INVALID_ARG = 1, /* NULL pointer, bad size, bad ordering, bad layout */
  SPS_ERR_RANGE = 2,       /* sizes inconsistent with each other or the plan */
  SPS_ERR_NOMEM = 3,       /* device or host allocation failed */
  SPS_ERR_DEVICE = 4,      /* a HIP runtime call or kernel failed */
  SPS_ERR_OVERFLOW = 5,    /* a sum could exceed its integer type */
  SPS_ERR_TRUNCATED = 6    /* sps_detect found more candidates than cap */
} sps_status;

/* Observation description (Sec. 2.3, Eq. KDM): channel centre frequencies,
 * the reference frequency the delays are measured from (the top of the band,
 * Sec. 2), the sampling time, and the trial DMs. */
typedef struct {
  int32_t nchan;          /* number of channels, >= 1 */
  const double *freq_mhz; /* host [nchan] channel centres in MHz, each in (0, fref_mhz]; copied */
  double fref_mhz;        /* reference frequency in MHz (arrival times are quoted here) */
  double tsamp_s;         /* sampling time in seconds, > 0 */
  int32_t ndm;            /* number of trial DMs, >= 1 */
  const double *dm;       /* host [ndm] trial DMs in pc cm^-3, each >= 0; copied */
} sps_obs_desc;

typedef struct sps_plan_s *sps_plan;

/* Creates a plan on the current HIP device: computes the integer delay table
 *   D[d][c] = floor(x + 1/2),  x = (K_DM * dm[d] / tsamp_s) * (1/f_c^2 - 1/f_ref^2)
 * with K_DM = 4.148808e3 s MHz^2 pc^-1 cm^3 (Eq. KDM; the paper prints the
 * unit as ms, which would be 10^3 too small) in IEEE double on the host, and
 * uploads it.  INVALID_ARG: NULL pointers, nchan/ndm < 1, tsamp_s <= 0,
 * a channel above fref_mhz or at a non-positive frequency, a negative DM.
 * OVERFLOW: a delay above 2^31 - 1 samples, or 255 * nchan >= 2^31.
 * NOMEM / DEVICE: allocation or upload failed.  *out is NULL on failure. */
sps_status sps_plan_create(const sps_obs_desc *desc, sps_plan *out);

/* Frees the plan and its device memory.  NULL is accepted.  The caller must
 * make sure no enqueued work still uses the plan. */
sps_status sps_plan_destroy(sps_plan plan);

/* Copies the delay table to host_out ([ndm][nchan] int32, row-major) when it
 * is not NULL, and the largest delay to *max_delay when that is not NULL. */
sps_status sps_plan_delays(sps_plan plan, int32_t *host_out, int32_t *max_delay);

/* Dedispersion flags. */
#define SPS_ZERO_PAD 1u /* allow nsamp_in < nout + max_delay: samples at or past
                           nsamp_in contribute zero (Eq. stage1's convention) */

/* Brute-force dedispersion (Sec. 2.3):
 *   Y[d][t] = sum_c X[c][t + D[d][c]],  t in [0, nout),
 * exact in unsigned 32-bit integers (every sum is at most 255 * nchan).
 *   X:        device uint8 [nchan][pitch], channel-major; only the first
 *             nsamp_in samples of each row are read, the rest of the row is
 *             padding.  X must be 16-byte aligned and pitch a multiple of 16
 *             (INVALID_ARG otherwise); the buffer holds nchan * pitch bytes.
 *   nsamp_in: valid samples per channel row, 0 <= nsamp_in <= pitch.
 *   Y:        device uint32 [ndm][nout], fully overwritten.
 *   nout:     output samples per DM row, 1 <= nout <= 2^31 - 1.
 *   flags:    0 requires nsamp_in >= nout + max_delay (RANGE otherwise), so
 *             every output is a full sum; SPS_ZERO_PAD relaxes it.
 * Output time index t is the arrival time at f_ref (Sec. 2).  Asynchronous. */
sps_status sps_dedisperse(sps_plan plan, const uint8_t *X, int64_t pitch, int64_t nsamp_in,
                          uint32_t *Y, int64_t nout, uint32_t flags, void *stream);

/* Boxcar matched-filter S/N over the DM-time plane (Sec. 1, step iii).
 * Per DM row d: med_d = lower median of Y[d][0..nout) (rank floor((n-1)/2)),
 * MAD_d = lower median of |Y[d][t] - med_d|, sigma_d = 1.4826 * MAD_d.
 * For each width w = widths[i] with t + w <= nout:
 *   S/N_w(t) = (sum_{k<w} Y[d][t+k] - w * med_d) / (sigma_d * sqrt(w)),
 * the numerator exact in integers, the scale in binary32.  Outputs:
 *   snr[d][t]    = max over fitting widths (binary32); 0 if MAD_d = 0;
 *   best_w[d][t] = index i of the smallest width attaining the maximum,
 *                  0xFF if no width fits (then snr is 0).
 *   Y:       device uint32 [ndm][nout] (the dedispersed plane).
 *   widths:  host int32 [nw], 1 <= nw <= 64, strictly ascending, widths[0] >= 1,
 *            widths[nw-1] <= nout (INVALID_ARG / RANGE otherwise).
 *   snr:     device float [ndm][nout];  best_w: device uint8 [ndm][nout].
 *   stats:   device int32 [ndm][2] receiving (med_d, MAD_d), or NULL.
 * OVERFLOW if widths[nw-1] * 255 * nchan >= 2^31.  Asynchronous. */
sps_status sps_boxcar_snr(sps_plan plan, const uint32_t *Y, int64_t nout,
                          const int32_t *widths, int32_t nw, float *snr, uint8_t *best_w,
                          int32_t *stats, void *stream);

/* One detected candidate (Sec. 2: DM, TOA referenced to the top of the band,
 * S/N, width). */
typedef struct {
  int32_t dm_idx; /* trial index d */
  int32_t width;  /* boxcar width in samples, widths[best_w[d][t]] */
  int64_t t_idx;  /* window start sample */
  float snr;      /* S/N at (d, t) */
  float reserved; /* 0 */
  double dm;      /* trial DM value, pc cm^-3 */
  double toa_s;   /* (t_idx + width / 2) * tsamp_s: window centre at f_ref */
} sps_candidate;

typedef struct {
  float threshold; /* keep tile maxima with S/N >= threshold; must be > 0 */
  int32_t tile_dm; /* tile height in DM trials, >= 1 */
  int64_t tile_t;  /* tile length in samples, >= 1; tile_dm * tile_t < 2^32 */
  int32_t nms_dm;  /* suppression radius in trials, >= 0 */
  int64_t nms_t;   /* suppression radius in samples, >= 0 */
} sps_detect_params;

/* Candidate detection on a boxcar S/N plane.  The plane is cut into tiles of
 * tile_dm x tile_t (the last ones ragged); each tile offers its maximum
 * (ties: smallest t, then smallest d) if it reaches the threshold.  Offers
 * are taken in order of S/N descending, then t, then d, and accepted unless
 * an accepted one lies within |dd| <= nms_dm and |dt| <= nms_t.
 *   snr, best_w: device planes as written by sps_boxcar_snr.
 *   widths/nw:   the same host width list.
 *   out:         host array of cap records (may be NULL when cap == 0),
 *                receiving the first min(n, cap) accepted in that order.
 *   n_found:     host, receives n, the number accepted.
 * Any number of tiles may reach the threshold.  Suppression radii larger
 * than the plane act as the plane's extent.  The plan keeps device scratch
 * of about 56 bytes per tile (allocated on first use, grown with the tile
 * count).  Returns SPS_ERR_TRUNCATED (after filling out) if n > cap.
 * Synchronises the stream. */
sps_status sps_detect(sps_plan plan, const float *snr, const uint8_t *best_w, int64_t nout,
                      const int32_t *widths, int32_t nw, const sps_detect_params *params,
                      sps_candidate *out, int32_t cap, int32_t *n_found, void *stream);

/* The search of one plane in one call: row statistics and boxcar S/N as in
 * sps_boxcar_snr, then candidates as in sps_detect, with the tile maxima
 * gathered by the boxcar pass itself (each boxcar workgroup reduces its
 * outputs to one key per tile and merges it atomically) instead of a
 * second pass over the S/N plane.  Same arguments, checks, results and
 * errors as sps_boxcar_snr followed by sps_detect on the same plan (Sec. 1
 * step iii; Sec. 2, candidate record); snr, best_w and stats receive the
 * same planes.  snr and best_w may both be NULL: then no S/N or width plane
 * is written (4 bytes of traffic per output instead of 13) and each tile's
 * key carries the width of its peak; the candidates are the same.  That
 * mode needs min(tile_dm, ndm) x min(tile_t, nout) <= 2^26 (else RANGE).
 * Uses the plan's detection scratch (grown on demand).  Synchronises the
 * stream. */
sps_status sps_search(sps_plan plan, const uint32_t *Y, int64_t nout, const int32_t *widths,
                      int32_t nw, float *snr, uint8_t *best_w, int32_t *stats,
                      const sps_detect_params *params, sps_candidate *out, int32_t cap,
                      int32_t *n_found, void *stream);

/* Statistics and boxcar S/N as in sps_boxcar_snr, but instead of the S/N
 * and width planes the pass writes the learned detector's input tiles
 * directly: the S/N of each whole tile of 512 trials x 4096 samples,
 * max-pooled over 2 trials x 8 samples, times scale, rounded to bfloat16
 * (nearest, ties to even) -- the tiles sps_cnn_pool_tile_grid makes from
 * the S/N plane, bit for bit.  tiles: device bf16 [ntiles][256][512] in
 * row-major tile order, ntiles = (ndm / 512) * (nout / 4096) (returned in
 * *ntiles if not NULL); a ragged rest of the plane makes no tile.  stats
 * as in sps_boxcar_snr.  Asynchronous. */
sps_status sps_boxcar_pool(sps_plan plan, const uint32_t *Y, int64_t nout, const int32_t *widths,
                           int32_t nw, int32_t *stats, float scale, uint16_t *tiles,
                           int64_t *ntiles, void *stream);

/* sps_detect for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, checks, kernels and results, but the detection
 * scratch is a fixed 4 MiB array in the library's device image, one copy
 * per device, held until the process ends, instead of plan memory grown
 * with hipMalloc.  It calls no hipMalloc, hipFree or other allocating
 * routine.  Holds at least 65,536 tiles (the scratch of ntiles tiles takes
 * about 56 bytes per tile); a plane that needs more returns SPS_ERR_RANGE
 * before anything is enqueued.  Every call on one device uses that device's
 * one copy: calls that overlap on a device (other streams, other threads)
 * race and must be serialised by the caller.  Synchronises the stream. */
sps_status sps_detect_noalloc(sps_plan plan, const float *snr, const uint8_t *best_w,
                              int64_t nout, const int32_t *widths, int32_t nw,
                              const sps_detect_params *params, sps_candidate *out, int32_t cap,
                              int32_t *n_found, void *stream);

/* Tiling of the dedispersion kernel, for tuning (sps_plan_create picks a
 * default).  m: output dwords per lane (odd), dpw: trials per wave, nw: waves
 * per workgroup, cs: channels per LDS slab, waves_per_eu: register budget
 * (0 = any compiled variant).  m == 0 selects the plain global-memory
 * kernel.  INVALID_ARG if the combination is not compiled in, RANGE if its
 * double-buffered LDS slab would exceed 160 KiB for this plan's delays. */
sps_status sps_plan_set_tiling(sps_plan plan, int32_t m, int32_t dpw, int32_t nw, int32_t cs,
                               int32_t waves_per_eu);
sps_status sps_plan_get_tiling(sps_plan plan, int32_t *m, int32_t *dpw, int32_t *nw, int32_t *cs,
                               int32_t *waves_per_eu, int32_t *lds_bytes);

/* ---- The paper's own dedispersion (Sec. 2.3) and pre-processing (Sec. 2.1-2.2) ---- */

/* Subband (two-stage) plan.  Fine grid DM_m = dm_lo + m dm_step (m < ndm),
 * coarse grid DM_j = dm_lo + j n0 dm_step.  Channels are split into nsub
 * contiguous subbands, subband s holding channels
 * [floor(s nchan / nsub), floor((s + 1) nchan / nsub)), represented by F_s
 * with 1/F_s^2 the mean of 1/f^2 over its channels (the paper allows "a
 * 1/f^2-weighted centre").  The plan is a superset of sps_plan_create's
 * (its fine delay table serves sps_dedisperse too) and adds:
 *   coarse delays  D_jc = round((K DM_j / t_samp)(1/f_c^2 - 1/f_ref^2))   Eq. (coarse_delay)
 *   residuals      R_ms = round((K (DM_m - DM_j(m)) / t_samp)(1/F_s^2 - 1/f_ref^2)),
 *                  j(m) = floor(m / n0)                                    Eq. (residual)
 * (round = half up).  INVALID_ARG / OVERFLOW as sps_plan_create, plus
 * n0 < 1, nsub outside [1, nchan], negative or non-finite DMs. */
typedef struct {
  int32_t nchan;
  const double *freq_mhz; /* host [nchan] channel centres, each in (0, fref_mhz]; copied */
  double fref_mhz;
  double tsamp_s;
  int32_t ndm;    /* fine trials */
  double dm_lo;   /* first trial DM */
  double dm_step; /* fine DM step */
  int32_t n0;     /* coarse step = n0 fine steps */
  int32_t nsub;   /* number of subbands */
} sps_subband_desc;
sps_status sps_subband_plan_create(const sps_subband_desc *desc, sps_plan *out);

/* Host copies of the subband tables: coarse_delays [ceil(ndm/n0)][nchan],
 * residuals [ndm][nsub], fsub [nsub] (MHz); each may be NULL.  *max_delay
 * receives the largest effective delay D_j(m)c + R_m,s(c). */
sps_status sps_subband_tables(sps_plan plan, int32_t *coarse_delays, int32_t *residuals,
                              double *fsub, int32_t *max_delay);

/* Two-stage subband dedispersion (Eq. stage1, Eq. stage2):
 *   I[j][s][u] = sum_{c in s} X[c][u + D_jc],  Y[m][t] = sum_s I[j(m)][s][t + R_ms],
 * samples past nsamp_in counting zero.  Equals brute force with the
 * effective delays D_j(m)c + R_m,s(c), and brute force itself when n0 = 1.
 * Arguments and flags as sps_dedisperse, with the effective max delay in the
 * strict-mode check.  The plan allocates nsub x ceil(ndm/n0) x (nout + max
 * R) x 4 bytes of device scratch on first use (and grows it).  Asynchronous. */
sps_status sps_dedisperse_subband(sps_plan plan, const uint8_t *X, int64_t pitch,
                                  int64_t nsamp_in, uint32_t *Y, int64_t nout, uint32_t flags,
                                  void *stream);

/* Zero-DM filter (Sec. 2.1 cites it; no formula is given).  Read as
 * subtraction of the DM = 0 series, the channel mean at each sample rounded
 * half up, m(t) = floor((sum_c X[c][t] + nchan/2) / nchan), about the 8-bit
 * mid-level:  Xo[c][t] = clip(X[c][t] - m(t) + 128, 0, 255).
 * X, Xo: device uint8 [nchan][pitch] / [nchan][pitch_out], 16-byte aligned,
 * pitches multiples of 16; Xo may equal X.  Asynchronous. */
sps_status sps_zero_dm(const uint8_t *X, int64_t pitch, int64_t nsamp, int32_t nchan, uint8_t *Xo,
                       int64_t pitch_out, void *stream);

/* Square-law downsampling by an integer factor N (Sec. 2.2):
 *   Xo[c][t] = min{ 255 sqrt(S) / sqrt(255 N), 255 },  S = sum_{k<N} X[c][tN + k],
 * rounded half up (exactly, in integers), for the full bins t < nsamp / N.
 * X: device uint8 [nchan][pitch]; Xo: device uint8 [nchan][pitch_out],
 * pitch_out >= nsamp / N.  1 <= nchan <= 65535.  Asynchronous. */
sps_status sps_downsample_sqrt(const uint8_t *X, int64_t pitch, int64_t nsamp, int32_t nchan,
                               int32_t factor, uint8_t *Xo, int64_t pitch_out, void *stream);

/* ---- Many filterbanks sharing one plan (beams of one receiver) ---- */

/* One filterbank of a batch and its outputs (all device pointers, caller-owned;
 * layouts as in sps_dedisperse / sps_boxcar_snr).  Beams may have different
 * lengths (nout, nsamp_in). */
typedef struct {
  const uint8_t *X; /* [nchan][pitch], 16-byte aligned, pitch % 16 == 0 */
  int64_t pitch;
  int64_t nsamp_in;
  uint32_t *Y;      /* [ndm][nout] */
  int64_t nout;     /* >= largest width */
  float *snr;       /* [ndm][nout], or NULL with best_w (see below) */
  uint8_t *best_w;  /* [ndm][nout], or NULL with snr */
  int32_t *stats;   /* [ndm][2] */
} sps_beam;

typedef struct sps_batch_s *sps_batch;

/* Fixes a batch: validates every beam as the single-filterbank calls would,
 * uploads the work description and allocates all scratch, so that running
 * the batch allocates nothing and never waits on the host.  The plan's
 * current tiling is used (call sps_plan_autotune / sps_plan_set_tiling
 * first); the plan must outlive the batch.  RANGE if the plan needs the
 * plain kernel.  Every beam's candidates read "none" until its first run.
 * Either every beam has snr and best_w or none has (INVALID_ARG otherwise):
 * without them the batch searches as sps_search does without planes (same
 * candidates, same tile size limit). */
sps_status sps_batch_create(sps_plan plan, int32_t nbeams, const sps_beam *beams,
                            const int32_t *widths, int32_t nw, const sps_detect_params *params,
                            uint32_t flags, sps_batch *out);
sps_status sps_batch_destroy(sps_batch batch);

/* Enqueues the whole search for every beam: one batched dedispersion
 * launch over all (beam, time tile, DM block) items, then batched row
 * statistics, boxcar S/N and detection (4 + 1 launches in total).  Makes no
 * allocation and no host synchronisation, so it may be captured into a HIP
 * graph.  Asynchronous. */
sps_status sps_batch_enqueue(sps_batch batch, void *stream);

/* As sps_batch_enqueue, replayed from a HIP graph captured on the first call
 * (and re-captured if the stream changes).  stream must not be NULL. */
sps_status sps_batch_launch_graph(sps_batch batch, void *stream);

/* Batch autotuner: times the batch's own batched dedispersion launch
 * over its beams with every compiled tiling that fits the plan (iters timed
 * launches each, HIP events, after one warm-up) and keeps the fastest for
 * this batch (the plan's tiling is unchanged).  Overwrites the beams' Y.
 * ms_out (optional) receives the mean time per tiling index (-1 where it
 * does not fit); *n_tried the number timed.  Allocates and frees the staged
 * tables it times; synchronises the stream; the next sps_batch_launch_graph
 * captures a new graph. */
sps_status sps_batch_autotune(sps_batch batch, int32_t iters, void *stream, float *ms_out,
                              int32_t *n_tried);

/* Tile mode: with tiles not NULL, every later enqueue or graph replay of
 * the batch runs dedispersion and statistics as before, then writes the
 * learned detector's input tiles straight from the boxcar pass (as
 * sps_boxcar_pool does for one plane) instead of the beams' S/N and width
 * planes and candidates: beam b's whole tiles follow those of beams < b in
 * tiles (device bf16 [ntiles][256][512]).  *ntiles (if not NULL) receives
 * the batch's tile count.  tiles NULL returns to the search mode.  A
 * change of mode discards the captured graph.  Must not overlap a run of
 * the batch. */
sps_status sps_batch_set_tiles(sps_batch batch, uint16_t *tiles, float scale, int64_t *ntiles);

/* Synchronises the stream and returns beam's candidates as sps_detect does
 * (same order, TRUNCATED / RANGE rules); INVALID_ARG in tile mode. */
sps_status sps_batch_candidates(sps_batch batch, int32_t beam, sps_candidate *out, int32_t cap,
                                int32_t *n_found, void *stream);

/* Every beam's candidates in one call (Sec. 2, candidate record): out is
 * host [nbeams][cap], beam b's first min(n_b, cap) candidates at out + b cap
 * in sps_detect's order; n_found is host [nbeams] and receives every n_b.
 * One gather launch and one copy into pinned memory the batch allocated at
 * creation bring back up to 512 records per beam, then one synchronisation
 * of the stream; a beam with more than 512 candidates to return takes its
 * own further copies.  Allocates nothing.  TRUNCATED (after filling) if any
 * n_b > cap; INVALID_ARG in tile mode. */
sps_status sps_batch_candidates_all(sps_batch batch, sps_candidate *out, int32_t cap,
                                    int32_t *n_found, void *stream);

/* Autotuner: times every compiled dedispersion tiling that fits the plan on
 * a probe of nout_probe output samples (iters timed runs each, HIP events,
 * after one warm-up) and keeps the fastest.  ms_out (optional) receives the
 * mean time per tiling index (-1 for tilings that do not fit), see
 * sps_tiling_describe; *n_tried the number timed.  For a subband plan whose
 * subbands are equal it also times stage 1 in one segmented launch against
 * one launch per subband on the same probe and keeps the faster form for
 * sps_dedisperse_subband (results are identical either way).  Allocates and
 * frees its probe buffers; synchronises the stream. */
sps_status sps_plan_autotune(sps_plan plan, int64_t nout_probe, int32_t iters, void *stream,
                             float *ms_out, int32_t *n_tried);
int32_t sps_tiling_count(void);
sps_status sps_tiling_describe(int32_t index, int32_t *m, int32_t *dpw, int32_t *nw, int32_t *cs,
                               int32_t *waves_per_eu);

/* Device microbenchmarks for the rates the kernels are measured against, on
 * HIP device `device`, written to rates[0 .. SPS_PROBE_COUNT-1]:
 *   rates[SPS_PROBE_VALU_ADD]  sustained v_add_u32 lane-ops per second,
 *   rates[SPS_PROBE_VALU_ADD3] sustained three-input adds (v_add3_u32) per second,
 *   rates[SPS_PROBE_VALU_PERM] sustained byte permutes (v_perm_b32) per second,
 *   rates[SPS_PROBE_LDS_READ]  sustained LDS read bytes per second
 *                              (16-byte lane-consecutive reads, no bank conflicts),
 *   rates[SPS_PROBE_LDS_READ32] the same with 4-byte reads.
 * The vector rates come from eight independent chains of the instruction on
 * every lane of 8192 workgroups of 256 threads.  The figures derived from
 * unit counts: 256 CUs x 64 lanes x 2 lane-ops per clock x 2.4 GHz =
 * 78.6e12/s (the lane rate behind the 157.3 TFLOP/s FP32 vector peak), which
 * two-operand ops approach and three-operand ops reach half of; LDS reads,
 * 256 B/clk/CU x 256 x 2.4 GHz = 157.3e12 B/s with 16-byte reads, half of
 * that with 4-byte reads.
 * Synchronous (own stream); allocates and frees 8 MB of device memory; about
 * 30 ms.  INVALID_ARG: rates NULL, n < SPS_PROBE_COUNT, or no such device;
 * DEVICE on a HIP error. */
enum { SPS_PROBE_VALU_ADD = 0, SPS_PROBE_VALU_ADD3 = 1, SPS_PROBE_VALU_PERM = 2,
       SPS_PROBE_LDS_READ = 3, SPS_PROBE_LDS_READ32 = 4, SPS_PROBE_COUNT = 5 };
sps_status sps_probe_peaks(int32_t device, double *rates, int32_t n);

/* ---- Streaming: many real-time filterbank streams on one GPU ---- */

/* A server searches admitted streams chunk by chunk.  Each stream keeps a
 * device ring of nchan x (O + chunk_len) bytes: the last O samples of the
 * previous chunk (the dispersion overlap of the time blocking in Sec. 2.3;
 * O = D_max rounded up to a multiple of 16), then the new chunk, so chunk k's
 * outputs are the dedispersed series at absolute samples
 * [k chunk_len - O, (k+1) chunk_len - O) of the stream (the overlap is zero
 * before chunk 0).  Worker w owns a HIP stream, a staging buffer for one
 * chunk, one plan per observing set-up and output planes sized for the
 * largest stream; streams of one set-up share its plans.  One chunk's
 * kernels run at a time; uploads of other chunks overlap them.  A chunk is
 * searched as sps_search does it; without an attached detector (which reads
 * the S/N plane) no S/N or width plane is written, where the stream's tiles
 * fit the packed tile keys. */
typedef struct sps_server_s *sps_server;

/* hbm_budget: device bytes the server may hold (rings, plans, planes);
 * 1 <= nworkers <= 16.  Uses the current device. */
sps_status sps_server_create(int64_t hbm_budget, int32_t nworkers, sps_server *out);
/* Waits for outstanding work and frees everything. */
sps_status sps_server_destroy(sps_server server);

/* Admits a stream: desc as for sps_plan_create, widths/nw and det as for
 * sps_boxcar_snr / sps_detect (checked here exactly as those calls check
 * them, so that no chunk fails for its parameters), chunk_len >= largest
 * width.  NOMEM (nothing allocated) when ring + new plans (with their
 * detection scratch) + plane growth would exceed the budget.
 * *stream_id numbers streams 0, 1, ... in admission order. */
sps_status sps_server_add_stream(sps_server server, const sps_obs_desc *desc,
                                 const int32_t *widths, int32_t nw, const sps_detect_params *det,
                                 int64_t chunk_len, int32_t *stream_id);
/* Device bytes accounted so far and the budget. */
sps_status sps_server_memory(sps_server server, int64_t *used, int64_t *budget);
/* Chunk length, overlap O (samples) and chunk duration (s) of a stream. */
sps_status sps_server_stream_info(sps_server server, int32_t stream_id, int64_t *chunk_len,
                                  int64_t *overlap, double *duration_s);

/* Searches the stream's next chunk now, on worker 0, and waits for it.
 * host: [nchan][src_pitch] bytes, first chunk_len of each row used (pinned
 * memory with src_pitch == chunk_len takes the fast linear upload).  Y_copy
 * (optional): device [ndm][chunk_len] that receives the dedispersed plane.
 * out/cap/n_found and TRUNCATED as in sps_detect.  n_cnn (optional, host)
 * receives the attached detector's count (sps_server_set_detector; 0 without
 * one).  Must not overlap sps_server_run. */
sps_status sps_server_push(sps_server server, int32_t stream_id, const uint8_t *host,
                           int64_t src_pitch, uint32_t *Y_copy, sps_candidate *out, int32_t cap,
                           int32_t *n_found, int32_t *n_cnn);

/* Source of a stream's chunks in sps_server_run: nsrc chunks of
 * [nchan][src_pitch] bytes back to back at host; chunk k of the run reads
 * source (first + k) % nsrc. */
typedef struct {
  const uint8_t *host;
  int64_t src_pitch;
  int32_t nsrc;
  int32_t first;
} sps_feed;

/* One searched chunk: times in seconds from the start of the run. */
typedef struct {
  int32_t stream;
  int32_t worker;
  int64_t index;    /* chunk number within the run */
  double arrival_s; /* scheduled arrival */
  double start_s;   /* a worker took it */
  double upload_s;  /* its samples were in the device ring */
  double compute_s; /* it held the compute lock (kernels start) */
  double end_s;     /* candidates on the host */
  int32_t n_cand;   /* candidates found (true count) */
  int32_t status;   /* sps_status of the chunk */
  int32_t n_cnn;    /* cells the attached detector flagged (0 without one) */
  int32_t reserved;
} sps_chunk_record;

/* Serves every admitted stream for run_s seconds of wall clock: stream i's
 * chunk k arrives at phase_i + (k+1) T_i / compression (T_i = chunk_len *
 * tsamp, phase_i = i T_i / (compression * nstreams)); arrivals after run_s are
 * not issued, and the call returns when every issued chunk is searched.
 * Workers take chunks in arrival order, a stream's chunks in sequence.
 * records (cap entries) receive one record per chunk in arrival order;
 * *n_records is the true count (TRUNCATED if above cap).  A chunk that fails
 * with SPS_ERR_DEVICE or SPS_ERR_NOMEM stops the run and that status is
 * returned; any other failure is kept in the chunk's record (status) and the
 * run goes on. */
sps_status sps_server_run(sps_server server, const sps_feed *feeds, double run_s,
                          double compression, sps_chunk_record *records, int32_t cap,
                          int32_t *n_records);

/* ---- Learned candidate detector (BF16 matrix-core CNN) ---- */

/* Tiles: a boxcar S/N plane max-pooled over windows of 2 trials x 8 samples,
 * multiplied by `scale` (binary32) and rounded to bfloat16 (nearest, ties to
 * even); a tile is 256 rows x 512 columns, stored as bfloat16 bit patterns
 * (uint16_t), row-major, tiles back to back.
 *
 * Network: six 3x3 convolutions (zero padding 1; strides 2,2,2,2,2,1;
 * channels 1->16->32->64->128->128->128), bias and ReLU each, then a 1x1
 * head with 3 outputs for every cell of an 8 x 16 grid (a cell covers 32 x
 * 32 tile pixels): objectness logit, row and column offset of the pulse
 * inside the cell in cell units.  3x3 weights are used as bfloat16,
 * activations and back-propagated signals are stored as bfloat16, every
 * product accumulates in FP32; head, loss and Adam are FP32.
 *
 * Parameters (FP32, sps_cnn_param_count() values) in this order: for each 3x3
 * layer its weights [cout][cin][3][3] then its biases [cout]; then the head
 * weights [3][128] and biases [3].
 *
 * Loss (mean over tiles): per cell, binary cross-entropy of the objectness
 * logit against the label (positive cells weighted pos_weight, default 32),
 * averaged over the 128 cells, plus lambda_box (default 1) times the squared
 * errors of both offsets at positive cells.
 * Labels: FP32 [n][3][8][16]: objectness (0/1), row offset, column offset.
 *
 * A network may be used from one stream at a time. */
typedef struct sps_cnn_s *sps_cnn;

typedef struct {
  int32_t tile;    /* tile index in the batch */
  int32_t cell_dm; /* cell row, 0..7 */
  int32_t cell_t;  /* cell column, 0..15 */
  float prob;      /* sigmoid of the objectness logit */
  float row;       /* predicted pulse row in the tile (0..256) */
  float col;       /* predicted pulse column in the tile (0..512) */
} sps_cnn_candidate;

int64_t sps_cnn_param_count(void);
/* Allocates the network for batches of up to max_batch tiles (<= 4096) on
 * the current device: parameters zero, Adam state zero. */
sps_status sps_cnn_create(int32_t max_batch, sps_cnn *out);
sps_status sps_cnn_destroy(sps_cnn net);
/* Host copies of all parameters / gradients (synchronous).  set_params also
 * resets the Adam state and step count. */
sps_status sps_cnn_set_params(sps_cnn net, const float *host);
sps_status sps_cnn_get_params(sps_cnn net, float *host);
/* Loss weights for the following loss_grad / train_step calls. */
sps_status sps_cnn_set_loss_weights(sps_cnn net, float pos_weight, float lambda_box);
sps_status sps_cnn_set_grads(sps_cnn net, const float *host);
sps_status sps_cnn_get_grads(sps_cnn net, float *host);
/* The bfloat16 ReLU output of 3x3 layer `layer` (0..5) for the first n tiles
 * of the last forward pass, NHWC [n][h][w][cout] (synchronous). */
sps_status sps_cnn_activations(sps_cnn net, int32_t layer, int32_t n, uint16_t *host);
/* The bfloat16 signal back-propagated to the output of 3x3 layer `layer`
 * (gradient of the loss w.r.t. its pre-activation, masked by a > 0) for the
 * first n tiles of the last sps_cnn_loss_grad, NHWC (synchronous).
 * sps_cnn_train_step keeps the signals of layers 1..5 but not layer 0's,
 * which no product reads. */
sps_status sps_cnn_signals(sps_cnn net, int32_t layer, int32_t n, uint16_t *host);

/* Pools the S/N plane snr (device FP32 [ndm][pitch], first nout used) into
 * tiles (device uint16 [ndm/2][nout/8]); only full windows.  Asynchronous. */
sps_status sps_cnn_pool_tiles(const float *snr, int64_t pitch, int32_t ndm, int64_t nout,
                              float scale, uint16_t *tiles, void *stream);
/* The whole plane cut into tiles (tile (i, j): trials [512 i, 512 i + 512),
 * samples [4096 j, 4096 j + 4096), pooled as sps_cnn_pool_tiles), written back
 * to back in row-major tile order to tiles (device; may be NULL when the count
 * is 0).  *ntiles = (ndm / 512) (nout / 4096): only whole tiles.
 * Asynchronous. */
sps_status sps_cnn_pool_tile_grid(const float *snr, int64_t pitch, int32_t ndm, int64_t nout,
                                  float scale, uint16_t *tiles, int64_t *ntiles, void *stream);
/* The batch size the network was created for (0 for NULL). */
int32_t sps_cnn_max_batch(sps_cnn net);

/* Attaches the learned detector (NULL detaches): after the boxcar S/N, every
 * chunk's plane is cut into whole tiles (sps_cnn_pool_tile_grid with scale)
 * and run through net; the number of cells with probability >= threshold is
 * reported (n_cnn of push and of the chunk records).  The tile buffer counts
 * against the budget (NOMEM if it does not fit).  The server uses net only
 * while it holds its compute lock; net must outlive the attachment and must
 * not be used elsewhere meanwhile.  Must not overlap sps_server_run or
 * sps_server_push. */
sps_status sps_server_set_detector(sps_server server, sps_cnn net, float threshold, float scale);

/* Forward pass of n tiles (device, 16-byte aligned); head (optional, device
 * FP32 [n][3][8][16]) receives the head outputs.  Every layer's activation
 * is kept (sps_cnn_activations reads them back).  Asynchronous. */
sps_status sps_cnn_forward(sps_cnn net, const uint16_t *tiles, int32_t n, float *head,
                           void *stream);
/* The same forward pass for inference: identical head outputs and layer
 * 1-5 activations, but layer 0 is computed inside layer 1's workgroups and
 * its activation (1 MB per tile) is not kept.  Asynchronous. */
sps_status sps_cnn_infer(sps_cnn net, const uint16_t *tiles, int32_t n, float *head,
                         void *stream);
/* Forward, loss and backward: gradients of the mean loss into the network's
 * gradient buffer; loss (optional, device FP32) receives the loss.
 * Asynchronous. */
sps_status sps_cnn_loss_grad(sps_cnn net, const uint16_t *tiles, const float *labels, int32_t n,
                             float *loss, void *stream);
/* One Adam step (with bias correction) from the gradient buffer.  Asynchronous. */
sps_status sps_cnn_adam(sps_cnn net, float lr, float beta1, float beta2, float eps,
                        void *stream);
/* sps_cnn_loss_grad then sps_cnn_adam(lr, 0.9, 0.999, 1e-8); layer 0's
 * back-propagated signal is not stored (see sps_cnn_signals). */
sps_status sps_cnn_train_step(sps_cnn net, const uint16_t *tiles, const float *labels, int32_t n,
                              float lr, float *loss, void *stream);
/* Forward pass, then every cell whose objectness probability is >= threshold
 * (0 < threshold < 1), in tile then cell order.  Synchronises the stream.
 * *n_found is the true count; TRUNCATED if above cap. */
sps_status sps_cnn_detect(sps_cnn net, const uint16_t *tiles, int32_t n, float threshold,
                          sps_cnn_candidate *out, int32_t cap, int32_t *n_found, void *stream);

/* Message for the last failed call on this thread ("" if none). */
const char *sps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPS_H */

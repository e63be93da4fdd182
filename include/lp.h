/*
 * lp.h -- C ABI of liblp.so, the MI355X (gfx950) hot path of the lunar
 * nanosecond-pulse pipeline of Winchen et al., "Realtime processing of
 * LOFAR data for the detection of nano-second pulses from the Moon"
 * (arXiv:1612.06592).
 *
 * Per block of station subband data the path is
 *   lp_beamform   -> tied-array beams (Sec. 3, first paragraph: each station
 *                    signal summed with a complex weight set by the station
 *                    position and the beam direction, 8 N_S FLOP per sample)
 *   lp_dedisperse -> ionospheric de-dispersion (Sec. 3: multiplication in the
 *                    frequency domain by an STEC-dependent complex weight,
 *                    repeated over trial STEC values)
 *   lp_synthesize -> time-domain synthesis from the polyphase-filtered
 *                    subbands (Sec. 2 and Sec. 3, PPF inversion), fused with
 *                    the Hilbert envelope and per-window peak finding
 *   lp_trigger    -> trigger list for the transient-buffer read-out (Sec. 2)
 * and lp_server_* / lp_stream_* run that chain for many concurrent
 * observation streams with their state resident on the device.
 *
 * Conventions (the paper leaves them open):
 *   - Subband k of the 1024-point critically sampled station PPF has RF
 *     centre f0 + k * fs / M (f0 = 100 MHz, fs = 200 MHz: second Nyquist
 *     zone with the spectral flip undone); a subband sample lasts M / fs.
 *   - Beam weight of input (station s, polarisation p) toward direction n:
 *     a_sp exp(-2 pi i frac(f_k (r_s . n) / c)), r_s in ENU metres,
 *     n = (cos el sin az, cos el cos az, sin el).
 *   - De-dispersion: overlap-save with N_fft = 4096, hop 2048 and a bulk
 *     delay of D = 1024 subband samples; bin q (signed q_s, RF frequency
 *     f_k + q_s fs / (M N_fft)) is multiplied by
 *     exp(-2 pi i [kappa T / (f_k + nu_q) + q_s D / N_fft]), kappa =
 *     e^2 / (8 pi^2 eps0 m_e) * 1e16 / c per TECU.
 *   - Synthesis: Z_m[n] = sum_k d_k[m] e^{+2 pi i k n / M} and
 *     z[mM + n] = sum_{t<16} g[tM + n] Z_{m-t}[n] with g = M h, h the
 *     Kaiser(beta)-windowed sinc prototype of the station PPF (sum h = 1).
 *     The real 5 ns series is 2 Re z and the analytic envelope |2 z|.
 *   - Trigger: sigma^2 = mean of (2 Re z)^2 over the block's valid samples;
 *     windows are the M-sample frames; a window fires when its envelope
 *     maximum exceeds k_sigma * sigma; a run of fired windows gives one
 *     trigger at its maximum; trials of one beam within M samples merge.
 *     The reported sample is the ADC index at the array origin:
 *     frame * M + n - M * 16 - D * M.  Frames whose stream index is below
 *     D + 16 (start-up of a fresh stream) never fire and are not in sigma.
 *
 * Memory: every data, state and output buffer is device memory owned by
 * the caller (e.g. torch tensors); the library never frees them.  Unless
 * stated otherwise arguments named *_state are read and updated in place
 * and are all-zero for a fresh stream.  Descriptors (lp_array, lp_band,
 * lp_dir, TEC lists) are host memory read during the call only.  Device
 * tables derived from descriptors (beam weights, chirp constants, synthesis
 * taps) are cached in the lp_ctx as "plans": a new plan's tables are written
 * asynchronously on the stream of the call that needs them (no device-wide
 * synchronisation), by default into memory the library allocates, or into
 * a caller buffer bound with lp_ctx_bind_const.  At most lp_ctx_plan_cache
 * plans (default 64) are kept beyond those in use; the least recently used
 * one is evicted (after waiting for the device) when a new one is made.
 *
 * Errors: nothing throws across the ABI.  Argument errors return
 * LP_EINVAL synchronously and leave every buffer untouched; the message is
 * available from lp_last_error() (thread-local).  Kernel launches are
 * asynchronous on the caller's hipStream_t (passed as void*, NULL = the
 * null stream); device faults surface at the caller's next
 * synchronisation.  Entry points taking a ctx are thread-safe for distinct
 * streams.
 */
#ifndef LP_H
#define LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lp_status;
#define LP_OK 0
#define LP_EINVAL (-1)   /* bad argument                                  */
#define LP_ENOMEM (-2)   /* device allocation failed                      */
#define LP_EAGAIN (-3)   /* does not fit now (serving admission)          */
#define LP_EHIP (-4)     /* HIP runtime error                             */
#define LP_ECLOSED (-5)  /* stream or server closed                       */
#define LP_ETIMEOUT (-6) /* nothing completed within the timeout          */

/* Sample types of the station subband input. */
#define LP_CI8 1  /* complex int8: (re, im) int8 pairs                     */
#define LP_CI16 2 /* complex int16: (re, im) int16 pairs                   */

/* Beamformer arithmetic. */
#define LP_FP32 0      /* FP32 inputs and weights on the vector ALUs       */
#define LP_FP16_MFMA 1 /* FP16 inputs and weights, FP32 accumulation on the
                          matrix cores                                     */

/* Fixed stream geometry of this library. */
#define LP_M 1024      /* PPF channels (subband sample = LP_M ADC samples) */
#define LP_TAPS 16     /* PPF taps per channel                              */
#define LP_NFFT 4096   /* de-dispersion FFT length                          */
#define LP_HOP 2048    /* de-dispersion hop; n_t must be a multiple of it   */
#define LP_DELAY 1024  /* de-dispersion bulk delay in subband samples       */

/* lp_dedisperse flags */
#define LP_DD_KEEP_TAIL 1 /* read the tail state but do not update it      */

typedef struct lp_ctx lp_ctx;

typedef struct {
  int32_t n_st;        /* stations                                         */
  int32_t n_pol;       /* polarisations per station (both summed per beam) */
  const double *enu_m; /* [n_st][3] station positions, ENU metres          */
  const float *gain;   /* [n_st * n_pol] real input gains, or NULL (= 1)   */
} lp_array;

typedef struct {
  int32_t n_sb;        /* number of selected subbands                      */
  const int32_t *k;    /* [n_sb] subband ids, strictly ascending, 1..511   */
  double f0_hz;        /* RF frequency of subband 0 (100e6)                */
  double fs_hz;        /* ADC sample rate (200e6)                          */
  int32_t M;           /* must be LP_M                                     */
  int32_t taps;        /* must be LP_TAPS                                  */
  double kaiser_beta;  /* prototype window parameter (9)                   */
} lp_band;

typedef struct {
  double az_rad; /* azimuth from North through East                         */
  double el_rad; /* elevation                                               */
} lp_dir;

typedef struct {
  int64_t sample; /* ADC index at the array origin (stream time)          */
  int32_t beam;
  int32_t tec;    /* index into the TEC trial list                         */
  float snr;      /* envelope / sigma at the trigger                       */
  float peak;     /* envelope at the trigger                               */
} lp_trig;

/* Thread-local message of the last failing call on this thread. */
const char *lp_last_error(void);
const char *lp_version(void);

/* Context on one HIP device: prototype taps, FFT twiddles and the cache of
 * beam-weight and chirp tables.  Returns LP_EHIP if the device is absent. */
lp_status lp_ctx_create(int32_t hip_device, lp_ctx **out);
void lp_ctx_destroy(lp_ctx *ctx);

/* Take plan tables from a caller buffer: device memory [bytes], 256-byte
 * aligned, that the caller keeps allocated until lp_ctx_destroy or the next
 * bind.  Cached plans are dropped first (after waiting for the device);
 * LP_EINVAL if a plan is in use (an open serving stream).  dev = NULL goes
 * back to library-allocated tables.  When a new plan does not fit, unused
 * plans are evicted; if it still does not fit the call that needed it
 * returns LP_ENOMEM.  (A C2-sized band needs about 5 MB per chirp plan,
 * 13 MB for a uniform grid of trials, and 0.2-12 MB per beam-weight plan.) */
lp_status lp_ctx_bind_const(lp_ctx *ctx, void *dev, size_t bytes);
/* Keep at most max_plans cached plans that no call or stream is using.    */
lp_status lp_ctx_plan_cache(lp_ctx *ctx, int32_t max_plans);
/* Cached plans, those in use, and their device bytes (any may be NULL).   */
lp_status lp_ctx_plan_stats(lp_ctx *ctx, int32_t *n_plans, int32_t *n_held,
                            size_t *device_bytes);

/* ---- sizing helpers (bytes of caller-allocated device buffers) -------- */
/* y of lp_beamform: cf32 [n_beams][n_sb][n_t]                              */
size_t lp_beam_bytes(int32_t n_beams, int32_t n_sb, int64_t n_t);
/* tail_state of lp_dedisperse: cf32 [n_beams][n_sb][LP_NFFT - LP_HOP]      */
size_t lp_dd_state_bytes(int32_t n_beams, int32_t n_sb);
/* d of lp_dedisperse: cf32 [n_beams][n_tec][n_sb][n_t]                     */
size_t lp_dd_bytes(int32_t n_beams, int32_t n_tec, int32_t n_sb, int64_t n_t);
/* hist_state of lp_synthesize: cf32 [n_series][n_sb][16]                   */
size_t lp_syn_state_bytes(int32_t n_series, int32_t n_sb);
/* cand of lp_synthesize / lp_trigger: per series and frame the envelope
 * maximum (f32) and its offset in the frame (i32), then per series and
 * 16-frame chunk the FP32 sum of (2 Re z)^2 over valid samples.          */
size_t lp_cand_bytes(int32_t n_series, int64_t n_t);
/* work of lp_trigger: per series room for every run a block of n_t windows
 * can hold (n_t / 2), about n_beams * n_tec * n_t * 8 bytes; 0 on invalid
 * sizes.                                                                   */
size_t lp_trigger_work_bytes(int32_t n_beams, int32_t n_tec, int64_t n_t);

/* ---- the hot path ------------------------------------------------------ */

/* Multi-beam beamformer (paper Sec. 3, beamforming paragraph).
 *   x : device, [n_sb][n_t][n_st][n_pol] complex int (dtype LP_CI8 or
 *       LP_CI16), re/im interleaved, inputs contiguous.
 *   y : device, cf32 [n_beams][n_sb][n_t] (lp_beam_bytes), overwritten.
 *   prec: LP_FP32 or LP_FP16_MFMA.  In FP16 with gains, each input's
 *       weights are divided by 2^e, e = ceil(log2 |gain|), and its samples
 *       multiplied by 2^e at conversion (a power of two: exact), so the FP16
 *       weights keep full precision; for LP_CI16 only factors below 1 move to
 *       the samples (32767 * 2 would leave the FP16 range) and the weights
 *       keep the rest (|w| <= 256).  Gains must be 0 or of magnitude in
 *       (2^-15, 2^8], else LP_EINVAL.  int8 and |int16| <= 2048 convert to
 *       FP16 exactly.
 * Requires n_st * n_pol <= 128, n_beams <= 64 per call, n_t % 128 == 0, and
 * a time row (n_st * n_pol complex samples) a multiple of 4 bytes; with
 * LP_FP16_MFMA a row of at most 256 bytes (int16 samples: n_st * n_pol
 * <= 64).  Else LP_EINVAL.                                                */
lp_status lp_beamform(lp_ctx *ctx, const lp_array *array, const lp_band *band,
                      const lp_dir *beams, int32_t n_beams, const void *x,
                      int32_t dtype, int64_t n_t, int32_t prec, void *y,
                      void *hip_stream);

/* ---- two-stage beamforming (Sec. 4, network paragraph) ---------------- */
/* When the station-side cluster cannot ship every station, it forms
 * preliminary beams from subsets of the stations and the processing cluster
 * forms the final beams from those.
 *   groups: group[st] in 0..n_groups-1 for every station (host memory, read
 *   during the call); every group non-empty; n_groups <= 32.               */
typedef struct {
  int32_t n_groups;
  const int32_t *group;  /* [n_st]                                          */
} lp_groups;

/* Stage 1 (station side): for group g and preliminary direction p, the
 * regular beam (lp_beamform's weights) over the group's stations only:
 *   y1[g * n_prelim + p][s][t] = sum_{st in g, pol} w(st, pol, s, n_p) x.
 * x, dtype, n_t, prec as for lp_beamform; y1 is cf32
 * [n_groups * n_prelim][n_sb][n_t] (lp_beam_bytes), n_groups * n_prelim
 * <= 64.  LP_EINVAL on bad groups or shapes.                               */
lp_status lp_beamform_groups(lp_ctx *ctx, const lp_array *array,
                             const lp_groups *groups, const lp_band *band,
                             const lp_dir *prelim, int32_t n_prelim,
                             const void *x, int32_t dtype, int64_t n_t,
                             int32_t prec, void *y1, void *hip_stream);

/* Stage 2 (processing side): final beam b from the preliminary beams of
 * every group towards the preliminary direction nearest to n_b (p(b):
 * largest n_p . n_b, lowest p on ties), re-phased by the group's phase
 * centre r_g (mean station position):
 *   y[b][s][t] = sum_g exp(-2 pi i frac(f_s r_g . (n_b - n_p(b)) / c))
 *                y1[g * n_prelim + p(b)][s][t]
 * (coefficients in FP64, applied in FP32).  y1 as written by
 * lp_beamform_groups; y is cf32 [n_beams][n_sb][n_t], n_beams <= 64, any
 * n_t > 0; 8-byte aligned buffers (with at most 8 groups, an even n_t and
 * 16-byte aligned y1 and y the kernel moves two samples per access).      */
lp_status lp_beamform_stage2(lp_ctx *ctx, const lp_array *array,
                             const lp_groups *groups, const lp_band *band,
                             const lp_dir *prelim, int32_t n_prelim,
                             const lp_dir *beams, int32_t n_beams,
                             const void *y1, int64_t n_t, void *y,
                             void *hip_stream);

/* Per-subband overlap-save de-dispersion at n_tec trial STEC values (paper
 * Sec. 3, dispersion paragraph).
 *   y    : device cf32 [n_beams][n_sb][n_t] (the beamformer output).
 *   tail : device cf32 state [n_beams][n_sb][2048]: the last 2048 samples of
 *          the previous block; updated unless flags has LP_DD_KEEP_TAIL.
 *   d    : device cf32 [n_beams][n_tec][n_sb][n_t] (lp_dd_bytes).  Output
 *          sample t corresponds to input time t - LP_DELAY.
 * n_t must be a positive multiple of LP_HOP; tec_tecu values in [0, 1000]. */
lp_status lp_dedisperse(lp_ctx *ctx, const lp_band *band,
                        const double *tec_tecu, int32_t n_tec, const void *y,
                        int32_t n_beams, int64_t n_t, void *tail,
                        int32_t flags, void *d, void *hip_stream);

/* Synthesis filterbank, envelope and per-window peaks (paper Sec. 2-3, PPF
 * inversion; this library uses the one-shot synthesis filterbank g = M h).
 *   d      : device cf32 [n_series][n_sb][n_t] (series = beam * n_tec + tec).
 *   frame0 : stream index of the block's first subband sample.
 *   hist   : device cf32 state [n_series][n_sb][16], updated.
 *   x_out  : device f32 [n_series][n_t * LP_M] real series 2 Re z, or NULL.
 *   cand   : device, lp_cand_bytes(n_series, n_t), overwritten.
 * n_t must be a positive multiple of LP_HOP, and one series' input must be
 * below 4 GiB with a row to spare ((n_sb + 1) * n_t * 8 < 2^32; the kernel
 * uses 32-bit offsets).                                                    */
lp_status lp_synthesize(lp_ctx *ctx, const lp_band *band, const void *d,
                        int32_t n_series, int64_t n_t, int64_t frame0,
                        void *hist, float *x_out, void *cand,
                        void *hip_stream);

/* De-dispersion and synthesis of one block with the de-dispersed subbands
 * held for one beam's group of trials only (Sec. 3: the STEC search repeats
 * de-dispersion and inversion per trial value).  lp_dedisperse's d holds
 * n_beams * n_tec * n_sb * n_t complex samples (28.7 GB for 7 beams x 32
 * trials x 244 subbands x 65536); here the caller's work holds trial_group
 * trials of one beam, and per beam and group of trials the two stages run
 * back to back on hip_stream into the block's candidate array.  Every group
 * transforms its hops forward again (more work for smaller groups).
 *   y, tail : as lp_dedisperse (tail updated once, by each beam's last
 *             group); hist, cand, frame0: as lp_synthesize for n_beams *
 *             n_tec series (series = beam * n_tec + trial).
 *   work    : device, >= lp_ddsyn_work_bytes(n_sb, n_t, min(trial_group,
 *             n_tec)), 16-byte aligned; nothing is kept in it between calls.
 * Outputs equal lp_dedisperse + lp_synthesize within the chirp rounding (a
 * group's first trial takes its exact chirp; later trials step from it).
 * Limits as both of those; trial_group >= 1, n_beams * n_tec <= 65535.   */
size_t lp_ddsyn_work_bytes(int32_t n_sb, int64_t n_t, int32_t trial_group);
lp_status lp_dedisperse_synthesize(lp_ctx *ctx, const lp_band *band,
                                   const double *tec_tecu, int32_t n_tec,
                                   const void *y, int32_t n_beams,
                                   int64_t n_t, int64_t frame0, void *tail,
                                   void *hist, void *cand,
                                   int32_t trial_group, void *work,
                                   size_t work_bytes, void *hip_stream);

/* Trigger rules over one block's candidates (paper Sec. 2: the trigger that
 * reads out the transient buffers).  Every run of every series is kept and
 * merged, so the list equals the rules' full result whatever its length.
 *   cand     : device, as written by lp_synthesize (series = beam * n_tec +
 *              trial, n_t frames each).
 *   frame0   : stream index of the block's first frame (start-up rule).
 *   out      : device lp_trig[cap], ordered by (beam, sample); only the first
 *              cap triggers are written.
 *   n_out    : device int32, the true number of triggers (may exceed cap).
 *   snr_out  : device f32 [n_beams][n_tec] peak envelope / sigma, or NULL.
 *   best_tec : device i32 [n_beams] argmax of snr_out (lowest on ties), or
 *              NULL.
 *   sigma_out: device f32 [n_beams][n_tec], or NULL.
 *   work     : device scratch of lp_trigger_work_bytes(n_beams, n_tec, n_t),
 *              16-byte aligned; no state is kept in it between calls.
 * Requires n_t a positive multiple of LP_HOP up to 2^20, n_tec <= 4096,
 * n_beams * n_tec <= 65535 and n_beams * n_tec * n_t / 2 < 2^31; else
 * LP_EINVAL.                                                               */
lp_status lp_trigger(lp_ctx *ctx, const void *cand, int32_t n_beams,
                     int32_t n_tec, int64_t n_t, int64_t frame0,
                     float k_sigma, lp_trig *out, int32_t cap, int32_t *n_out,
                     float *snr_out, int32_t *best_tec, float *sigma_out,
                     void *work, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lp_trigger
 * with its workspace in a fixed device array of LP_TRIGGER_SCRATCH_BYTES
 * that the library holds on every device it runs on until the process ends
 * (its address is taken once per device by lp_ctx_create).  Arguments,
 * limits and results as lp_trigger, minus `work`; the call allocates
 * nothing.  LP_EINVAL when lp_trigger_work_bytes(n_beams, n_tec, n_t)
 * exceeds LP_TRIGGER_SCRATCH_BYTES (e.g. 61 beams x 1 trial x 32768 samples
 * needs 12 MB, 7 x 32 x 65536 needs 88 MB).  All calls on one device share
 * the array: calls that may overlap on the device (different streams, or
 * threads without ordering) race and must be serialised by the caller.   */
#define LP_TRIGGER_SCRATCH_BYTES ((size_t)128 << 20)
lp_status lp_trigger_noalloc(lp_ctx *ctx, const void *cand, int32_t n_beams,
                             int32_t n_tec, int64_t n_t, int64_t frame0,
                             float k_sigma, lp_trig *out, int32_t cap,
                             int32_t *n_out, float *snr_out, int32_t *best_tec,
                             float *sigma_out, void *hip_stream);

/* ---- plain FP32 comparator ------------------------------------------- */
/* The same de-dispersion and synthesis arithmetic organised the
 * straightforward way: every intermediate (overlap-save buffers, spectra,
 * each radix-2 FFT pass through global memory, filtered series, envelope,
 * real series) is a full array in device memory and every step is its own
 * kernel.  Arguments and outputs as lp_dedisperse / lp_synthesize (equal to
 * FP32 rounding); `work` is device scratch of work_bytes, at least
 * lp_plain_work_bytes (beams / series are processed in groups that fit).
 * This is the baseline against which the fused kernels are measured. */
size_t lp_plain_work_bytes(int32_t n_beams, int32_t n_tec, int32_t n_sb,
                           int64_t n_t);
lp_status lp_dedisperse_plain(lp_ctx *ctx, const lp_band *band,
                              const double *tec_tecu, int32_t n_tec,
                              const void *y, int32_t n_beams, int64_t n_t,
                              void *tail, int32_t flags, void *d, void *work,
                              size_t work_bytes, void *hip_stream);
lp_status lp_synthesize_plain(lp_ctx *ctx, const lp_band *band, const void *d,
                              int32_t n_series, int64_t n_t, int64_t frame0,
                              void *hist, float *x_out, void *cand, void *work,
                              size_t work_bytes, void *hip_stream);

/* ---- PPF inversion by LSMR (Sec. 3, "Computing requirements") ---------- */
/* The paper recovers the 5 ns signal by solving the sparse system H x = y
 * for the filtered subband data with the iterative LSMR method (Fong &
 * Saunders 2011), about 25 iterations.  H is the station's analysis
 * polyphase filterbank (prototype h: Kaiser-windowed sinc, band->kaiser_beta,
 * M = 1024, 16 taps) restricted to the subbands band->k:
 *   y_s[m] = sum_{l < 16384} h[l] exp(+2 pi i k_s l / 1024) x[1024 m + 1023 - l]
 * for output frames m = 0 .. n_frames - 1 of a real series x of
 * F = n_frames - 15 frames (1024 F samples; zero outside), so frame m of y
 * sees frames m - 15 .. m of x.
 * Layouts (device memory, caller-owned): y and d are complex float
 * [n_series][n_sb][n_frames] (the layout lp_dedisperse writes: series =
 * beam * n_tec + trial); x is float [n_series][F * 1024], time order.
 * n_frames in [16, 2^19] (the kernels address one series with 32-bit
 * offsets).  All calls are asynchronous on hip_stream.                     */

/* y = H x (the analysis filterbank; also a station-PPF simulator).        */
lp_status lp_ppf_analyze(lp_ctx *ctx, const lp_band *band, const float *x,
                         int32_t n_series, int64_t n_frames, void *y,
                         void *hip_stream);
/* x = H^T y, the real adjoint (x real, y complex, inner product Re <a, b>). */
lp_status lp_ppf_adjoint(lp_ctx *ctx, const lp_band *band, const void *y,
                         int32_t n_series, int64_t n_frames, float *x,
                         void *hip_stream);
/* Workspace of lp_ppf_invert (0 on invalid sizes).                         */
size_t lp_ppf_work_bytes(int32_t n_sb, int32_t n_series, int64_t n_frames);
/* n_iter LSMR iterations from x_0 = 0 with no damping, per series, in FP32
 * vectors with FP64 scalar recurrences; stops changing x once the
 * bidiagonalisation ends (alpha or beta zero; y = 0 gives x = 0).
 *   x      out, [n_series][F * 1024]
 *   anorm  out or NULL, double [n_series][n_iter + 1]: ||H^T r_k|| for
 *          k = 0 .. n_iter as LSMR's recurrence gives it (|zetabar_{k+1}|)
 *   rnorm  out or NULL, double [n_series]: ||y - H x|| computed from x
 *          (one more application of H)
 *   work   device, >= lp_ppf_work_bytes(), 256-byte aligned; no state is
 *          kept in it between calls.
 * LP_EINVAL on NULL or misaligned buffers, bad sizes or a short workspace. */
lp_status lp_ppf_invert(lp_ctx *ctx, const lp_band *band, const void *y,
                        int32_t n_series, int64_t n_frames, int32_t n_iter,
                        float *x, double *anorm, double *rnorm, void *work,
                        size_t work_bytes, void *hip_stream);

/* ---- station simulator (Sec. 2: 5 ns sampling and the station PPF;
 *      Sec. 5: the simulation chain's PPF module) ----------------------- */
typedef struct {
  uint64_t seed;        /* Philox4x32-10 key: (seed mod 2^32, seed div 2^32) */
  int32_t n_in;         /* inputs (stations x polarisations)                */
  int32_t noise_words;  /* R in 0..256: noise variance 8 R ADC units^2      */
  int32_t adc_bits;     /* codes saturate to [-2^(b-1), 2^(b-1) - 1], 2..16 */
} lp_sim_cfg;

/* ADC codes of every input for absolute samples n0 .. n0 + n_samp - 1:
 *   noise_i[n] = sum_{r < R} (popcount(w_r) - 16)
 * with w_r the words of Philox4x32-10 (Salmon et al. 2011) under the key and
 * the counter (n mod 2^32, n div 2^32, i, r div 4) (word r mod 4), so any
 * split of the sample range gives the same codes; plus, if pulse is not
 * NULL, rint (half to even) of pulse[i][n - pulse_n0] for n in [pulse_n0,
 * pulse_n0 + pulse_len); then saturated.  pulse: device float
 * [n_in][pulse_len]; adc: device int16 [n_in][n_samp].                      */
lp_status lp_sim_adc(lp_ctx *ctx, const lp_sim_cfg *cfg, int64_t n0,
                     int64_t n_samp, const float *pulse, int64_t pulse_n0,
                     int64_t pulse_len, int16_t *adc, void *hip_stream);

/* The station polyphase filterbank (prototype h of band->kaiser_beta,
 * M = 1024, 16 taps) of every input's ADC stream, for the subbands band->k:
 *   y_s[m] = sum_{l < 16384} h[l] exp(+2 pi i k_s l / 1024)
 *            adc[1024 (m + 16) - 1 - l]
 * for output frames m = 0 .. n_frames - 1 (adc holds 15 frames of history
 * before them: [n_in][(n_frames + 15) * 1024] int16), times scale, rounded
 * half to even and saturated to the int8 or int16 range (dtype LP_CI8 or
 * LP_CI16), written as the beamformer's input x [n_sb][n_frames][n_in]
 * complex.  n_in <= 128, n_frames <= 2^19 - 30.  work: device, >=
 * lp_station_work_bytes().  (n_in a multiple of 8 for LP_CI8, of 4 for
 * LP_CI16, with 16-byte aligned x and work, takes 16-byte stores.)          */
size_t lp_station_work_bytes(int32_t n_in, int32_t n_sb, int64_t n_frames);
lp_status lp_station_ppf(lp_ctx *ctx, const lp_band *band, const int16_t *adc,
                         int32_t n_in, int64_t n_frames, float scale,
                         int32_t dtype, void *x, void *work,
                         size_t work_bytes, void *hip_stream);

/* ---- serving: concurrent observation streams ------------------------- */
/* A persistent request loop (one host thread) runs the four stages for many
 * observation streams.  Each open stream keeps its overlap-save tail and
 * synthesis history resident in a caller-provided device arena; blocks are
 * admitted as slots and arena space free up, split into hop-aligned chunks,
 * and the next chunk is always taken from the admitted block with the
 * earliest deadline.  Each stream has its own HIP stream, so the chunks of
 * different streams overlap on the device.  Results are bitwise identical
 * to running the same blocks through lp_beamform .. lp_trigger directly.
 * The arena is carved by the server (first fit, 256-byte aligned); the
 * caller keeps it allocated until lp_server_destroy returns. */

typedef struct lp_server lp_server;

typedef struct {
  lp_array array;        /* copied at open                                 */
  lp_band band;          /* copied at open                                 */
  const lp_dir *beams;   /* [n_beams], copied at open                      */
  int32_t n_beams;       /* 1..64                                          */
  const double *tec_tecu;/* [n_tec], copied at open                        */
  int32_t n_tec;
  int32_t dtype;         /* LP_CI8 or LP_CI16                              */
  int32_t prec;          /* LP_FP32 or LP_FP16_MFMA                        */
  float k_sigma;         /* trigger threshold in sigma (6)                 */
  int64_t max_n_t;       /* longest block this stream will submit          */
  int32_t trig_cap;      /* triggers returned per block (0 = 1024)         */
  double deadline_s;     /* per-block latency budget; 0 = the 5 s transient
                            buffer minus the block's duration              */
} lp_stream_cfg;

typedef struct {
  int32_t stream;          /* id from lp_stream_open                        */
  int32_t status;          /* LP_OK, LP_ECLOSED (dropped at close), LP_EHIP */
  uint64_t tag;            /* the submit's tag                              */
  int64_t n_t;             /* block length (subband samples)                */
  int64_t frame0;          /* stream index of the block's first sample      */
  int32_t n_trig;          /* number of triggers (may exceed trig_cap)      */
  int32_t n_beams, n_tec;
  const lp_trig *trig;     /* host, min(n_trig, trig_cap) entries          */
  const float *snr;        /* host [n_beams][n_tec] peak envelope / sigma  */
  const int32_t *best_tec; /* host [n_beams]                                */
  int64_t submit_ns;       /* host steady clock at submit                   */
  int64_t done_ns;         /* host steady clock when the loop saw it done   */
  int64_t latency_ns;      /* done_ns - submit_ns                           */
  int64_t deadline_ns;     /* the block's latency budget                    */
} lp_result;

#define LP_SUBMIT_RESET 1  /* zero the stream state first (fresh stream)  */

/* Bytes of arena a stream keeps while open (state + chunk buffers) and
 * that one of its blocks of n_t samples holds while in flight.            */
size_t lp_stream_resident_bytes(const lp_stream_cfg *cfg, int64_t chunk_t);
size_t lp_block_bytes(const lp_stream_cfg *cfg, int64_t n_t);

/* chunk_t: samples per subband processed per chunk (multiple of LP_HOP;
 * 0 = 8192).  max_slots: blocks in flight at once (0 = 16). */
lp_status lp_server_create(lp_ctx *ctx, void *arena_dev, size_t arena_bytes,
                           int32_t max_slots, int64_t chunk_t,
                           lp_server **out);
/* A server whose executor only models time (ns_per_sample per station-beam
 * sample on one in-order device queue) and computes nothing: the request
 * loop, admission and scheduling run exactly as in the real server.  For
 * tests without a GPU; results have no triggers. */
lp_status lp_server_create_sim(double ns_per_sample, size_t arena_bytes,
                               int32_t max_slots, int64_t chunk_t,
                               lp_server **out);
/* LP_EAGAIN if the stream's resident bytes do not fit in the arena now. */
lp_status lp_stream_open(lp_server *srv, const lp_stream_cfg *cfg,
                         int32_t *id);
/* Queue a block: device memory [n_sb][n_t][n_st][n_pol] complex ints that
 * stays valid and unchanged until its result is polled.  Returns at once;
 * LP_EINVAL for a bad length (not a positive multiple of LP_HOP, or above
 * max_n_t), LP_ECLOSED if the stream is closing. */
lp_status lp_stream_submit(lp_server *srv, int32_t id, const void *block,
                           int64_t n_t, uint64_t tag, int32_t flags);
/* Wait up to timeout_us for results; returns up to cap of them in
 * completion order.  The arrays they point to stay valid until the next
 * lp_stream_poll on this server.  LP_ETIMEOUT if none arrived. */
lp_status lp_stream_poll(lp_server *srv, lp_result *out, int32_t cap,
                         int32_t *n, int32_t timeout_us);
/* Blocks already admitted finish; blocks still queued are returned with
 * status LP_ECLOSED; the stream's arena space is released afterwards. */
lp_status lp_stream_close(lp_server *srv, int32_t id);
/* Finishes admitted blocks, drops queued ones, stops the loop. */
void lp_server_destroy(lp_server *srv);
/* Aggregate counters: blocks done, chunks issued, admission waits. */
lp_status lp_server_stats(lp_server *srv, int64_t *blocks_done,
                          int64_t *chunks_issued, int64_t *admit_waits);

#ifdef __cplusplus
}
#endif
#endif

/*
 * lpo.h -- plain FP64 CPU oracle for the lunar ns-pulse hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant with the GPU library under
 * paper_1612_06592_amd/ and must never be used as a fallback for it.
 *
 * What it computes follows Winchen et al., "Realtime processing of LOFAR
 * data for the detection of nano-second pulses from the Moon"
 * (arXiv:1612.06592):
 *   Sec. 3 "Computing Requirements", beamforming paragraph  -> lpo_beamform
 *   Sec. 3, dispersion paragraph (STEC-dependent complex weight in the
 *           frequency domain, N-point radix-2 FFT)           -> lpo_dedisperse
 *   Sec. 2 / Sec. 3, PPF inversion (synthesis of the ns-resolution signal
 *           from the polyphase-filtered subbands)            -> lpo_synthesize
 *   Sec. 2, trigger for the transient-buffer read-out       -> lpo_detect,
 *                                                              lpo_trigger
 * The paper leaves the PPF parameters, the frequency mapping, the
 * overlap-save geometry and the trigger statistic open; each function
 * below states the reading it implements.
 *
 * Complex numbers are C99 `double complex` (interleaved re, im in memory).
 * All arrays are caller-owned host memory.
 */
#ifndef LPO_H
#define LPO_H

#include <complex.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* First-order ionospheric dispersion constant kappa = K_ion * 1e16 / c in
 * s^-1 per TECU, with K_ion = e^2 / (8 pi^2 eps0 m_e) from CODATA 2018.
 * The ionospheric phase of frequency f at slant TEC T (TECU) is
 * 2 pi kappa T / f radians; its group delay is kappa T / f^2 seconds. */
double lpo_kappa(void);
double lpo_speed_of_light(void);

/* Number of OpenMP threads the oracle uses. */
int lpo_threads(void);
void lpo_set_threads(int n);

/* In-place radix-2 FFT of length n (a power of two).
 * inverse = 0: X_q = sum_n x_n exp(-2 pi i q n / N)
 * inverse = 1: x_n = (1/N) sum_q X_q exp(+2 pi i q n / N)               */
void lpo_fft(long n, double complex *x, int inverse);

/* Modified Bessel function of the first kind, order 0, power series. */
double lpo_bessel_i0(double x);

/* Analysis prototype filter (Kaiser-windowed sinc), L = M * P taps:
 *   w[l] = I0(beta sqrt(1 - (2l/(L-1) - 1)^2)) / I0(beta)
 *   h[l] = w[l] sinc((l - (L-1)/2) / M),  sinc(x) = sin(pi x)/(pi x)
 * normalised so that sum_l h[l] = 1.                                      */
void lpo_prototype(int M, int P, double beta, double *h);

/* Analysis polyphase filterbank (the station PPF, used by the oracle's own
 * invariant tests only):
 *   y_k[m] = sum_{l=0}^{L-1} h[l] exp(+2 pi i k l / M) x[m M - l]
 * for frames m = m0 .. m0+n_frames-1 and the n_ch channels ch[].  x[n] is
 * taken as zero outside 0 <= n < n_x.  y is [n_ch][n_frames].            */
void lpo_analysis(int M, int P, const double *h, long n_x,
                  const double complex *x, long m0, long n_frames, int n_ch,
                  const int *ch, double complex *y);

/* Multi-beam (tied-array) beamformer.  For beam b, subband s with RF
 * centre f = f0 + k[s] * fs / M, and input (station st, polarisation p):
 *   w = a_{st,p} exp(-2 pi i frac(f (r_st . n_b) / c))
 *   y[b][s][t] = sum_{st,p} w * x[s][t][st][p]
 * r_st are ENU station positions in metres, n_b = (cos el sin az,
 * cos el cos az, sin el).  x holds (re, im) pairs laid out
 * [n_sb][n_t][n_st][n_pol][2] (integer samples are exact in FP64);
 * gain may be NULL (all ones).
 * y is [n_beams][n_sb][n_t].                                             */
void lpo_beamform(int n_st, int n_pol, const double *enu, const double *gain,
                  int n_sb, const int *k, double f0, double fs, int M,
                  int n_beams, const double *az_el, long n_t,
                  const double *x, double complex *y);

/* Dedispersion chirp of one subband for one slant TEC value, length n_fft:
 *   C_q = exp(-2 pi i [frac(kappa T / (f_k + nu_q)) + q_s D / n_fft])
 * with q_s the signed bin (q for q < n_fft/2, else q - n_fft) and
 * nu_q = q_s * df / n_fft (df = subband sample rate).                     */
void lpo_chirp(double f_k, double tec, int n_fft, int delay, double df,
               double complex *c);

/* Overlap-save dedispersion of every (beam, subband) series at every TEC
 * trial.  Per hop h the buffer u = [hist previous samples | hop new
 * samples] (hist = n_fft - hop; before the stream start the previous
 * samples come from `tail`, zero for a fresh stream), U = FFT(u),
 * v = IFFT(U * C_j), and d[..][h*hop + i] = v[hist + i], i < hop.
 * y: [n_beams][n_sb][n_t]; tail: [n_beams][n_sb][hist] (updated);
 * d: [n_beams][n_tec][n_sb][n_t].  n_t must be a multiple of hop.
 * Returns 0, or -1 on bad arguments.                                      */
int lpo_dedisperse(int n_sb, const int *k, double f0, double fs, int M,
                   int n_tec, const double *tec, int n_fft, int hop,
                   int delay, int n_beams, long n_t, const double complex *y,
                   double complex *tail, double complex *d);

/* Synthesis filterbank (one-shot inverse of the PPF).  Per series and
 * frame m:
 *   Z_m[n] = sum_{s} d_s[m] exp(+2 pi i k[s] n / M),   n = 0..M-1
 *   z[m M + n] = sum_{t=0}^{P-1} g[t M + n] Z_{m-t}[n],  g = M h
 * Frames before the block come from hist ([n_series][P-1][n_sb], the last
 * P-1 frames of the previous block, zero for a fresh stream; updated).
 * d: [n_series][n_sb][n_t]; z: [n_series][n_t * M].                       */
void lpo_synthesize(int M, int P, const double *h, int n_sb, const int *k,
                    int n_series, long n_t, const double complex *d,
                    double complex *hist, double complex *z);

/* Envelope statistics of one block per series.  e[n] = |2 z[n]|,
 * xr[n] = 2 Re z[n].  Frame m of the block is valid when frame0 + m >=
 * warm (warm = D + P frames of start-up from the stream origin).
 *   sigma = sqrt(mean of xr^2 over valid samples)  (0 if none)
 *   wmax[m], warg[m] = max of e over the M samples of frame m and the
 *   lowest block sample index m*M + n attaining it.                       */
void lpo_detect(int M, long n_t, long frame0, long warm, int n_series,
                const double complex *z, double *sigma, double *wmax,
                int64_t *warg);

typedef struct {
  int64_t sample; /* ADC index at the array origin                         */
  int32_t beam;
  int32_t tec;    /* trial index                                           */
  double snr;     /* e / sigma at the trigger                              */
  double peak;    /* e at the trigger                                      */
} lpo_trig;

/* Trigger rules.  Series index = beam * n_tec + tec.  A valid window m
 * fires when wmax > k_sigma * sigma (strict, sigma > 0).  Each maximal run
 * of consecutive fired windows gives one trigger at the run's largest
 * wmax (earliest on ties).  Its sample is frame0*M + warg - M*P - D*M.
 * Per beam, triggers of all trials are sorted by (sample, trial) and
 * chained while consecutive samples differ by at most M; each chain keeps
 * its highest snr (lowest trial, then lowest sample on ties).  Output is
 * ordered by (beam, sample).  snr_peak[b][j] = max valid wmax / sigma;
 * best_tec[b] = argmax_j snr_peak (lowest j on ties).  Returns the total
 * number of triggers (only the first `cap` are written).                 */
long lpo_trigger(int M, int P, int D, long n_t, long frame0, long warm,
                 int n_beams, int n_tec, const double *sigma,
                 const double *wmax, const int64_t *warg, double k_sigma,
                 long cap, lpo_trig *out, double *snr_peak, int *best_tec);

#ifdef __cplusplus
}
#endif
#endif

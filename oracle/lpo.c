/*
 * lpo.c -- plain FP64 CPU oracle for the lunar ns-pulse hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see lpo.h).  Every routine is the definition
 * written out with plain loops; the only "library" step is the radix-2
 * FFT below, itself checked against a brute-force DFT by the tests.
 * OpenMP only splits independent (beam, subband, trial, series) units
 * across threads; no unit's arithmetic depends on the thread count.
 */
#include "lpo.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* CODATA 2018 exact / recommended values. */
#define LPO_C 299792458.0           /* speed of light, m/s                 */
#define LPO_QE 1.602176634e-19      /* elementary charge, C                */
#define LPO_EPS0 8.8541878128e-12   /* vacuum permittivity, F/m            */
#define LPO_ME 9.1093837015e-31     /* electron mass, kg                   */

double lpo_speed_of_light(void) { return LPO_C; }

double lpo_kappa(void) {
  /* K_ion = e^2 / (8 pi^2 eps0 m_e) [m^3 s^-2]; 1 TECU = 1e16 m^-2.  The
   * ionospheric phase is 2 pi K_ion STEC / (c f); in cycles that is
   * (K_ion 1e16 / c) T / f. */
  double k_ion = LPO_QE * LPO_QE / (8.0 * M_PI * M_PI * LPO_EPS0 * LPO_ME);
  return k_ion * 1e16 / LPO_C;
}

int lpo_threads(void) { return omp_get_max_threads(); }

/* Thread count of later parallel loops (timing on one or more cores). */
void lpo_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* ------------------------------------------------------------------ FFT */

void lpo_fft(long n, double complex *x, int inverse) {
  /* Bit-reversal permutation. */
  for (long i = 1, j = 0; i < n; i++) {
    long bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double complex t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
  /* Radix-2 decimation-in-time butterflies; each twiddle is evaluated
   * directly from its angle (no recurrences). */
  double sgn = inverse ? 2.0 : -2.0;
  for (long len = 2; len <= n; len <<= 1) {
    long half = len >> 1;
    for (long s = 0; s < half; s++) {
      double ang = sgn * M_PI * (double)s / (double)len;
      double complex w = cos(ang) + I * sin(ang);
      for (long i = s; i < n; i += len) {
        double complex u = x[i];
        double complex v = x[i + half] * w;
        x[i] = u + v;
        x[i + half] = u - v;
      }
    }
  }
  if (inverse) {
    double sc = 1.0 / (double)n;
    for (long i = 0; i < n; i++) x[i] *= sc;
  }
}

/* ------------------------------------------------------------ prototype */

double lpo_bessel_i0(double x) {
  /* I0(x) = sum_m ((x/2)^m / m!)^2 */
  double q = 0.25 * x * x, term = 1.0, sum = 1.0;
  for (int m = 1; m < 500; m++) {
    term *= q / ((double)m * (double)m);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

void lpo_prototype(int M, int P, double beta, double *h) {
  long L = (long)M * P;
  double i0b = lpo_bessel_i0(beta);
  double sum = 0.0;
  for (long l = 0; l < L; l++) {
    double r = 2.0 * (double)l / (double)(L - 1) - 1.0;
    double a = 1.0 - r * r;
    double w = lpo_bessel_i0(beta * sqrt(a > 0.0 ? a : 0.0)) / i0b;
    double xs = ((double)l - 0.5 * (double)(L - 1)) / (double)M;
    double sinc = (xs == 0.0) ? 1.0 : sin(M_PI * xs) / (M_PI * xs);
    h[l] = w * sinc;
    sum += h[l];
  }
  for (long l = 0; l < L; l++) h[l] /= sum;
}

/* ---------------------------------------------------------- analysis PFB */

void lpo_analysis(int M, int P, const double *h, long n_x,
                  const double complex *x, long m0, long n_frames, int n_ch,
                  const int *ch, double complex *y) {
  long L = (long)M * P;
  double complex *rot = malloc(sizeof(double complex) * M);
  for (int r = 0; r < M; r++) {
    double ang = 2.0 * M_PI * (double)r / (double)M;
    rot[r] = cos(ang) + I * sin(ang); /* exp(+2 pi i r / M) */
  }
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int c = 0; c < n_ch; c++) {
    for (long i = 0; i < n_frames; i++) {
      long k = ch[c];
      long m = m0 + i;
      double complex acc = 0.0;
      for (long l = 0; l < L; l++) {
        long n = m * M - l;
        if (n < 0 || n >= n_x) continue;
        acc += h[l] * rot[(k * l) % M] * x[n];
      }
      y[(long)c * n_frames + i] = acc;
    }
  }
  free(rot);
}

/* ------------------------------------------------------------ beamform */

void lpo_beamform(int n_st, int n_pol, const double *enu, const double *gain,
                  int n_sb, const int *k, double f0, double fs, int M,
                  int n_beams, const double *az_el, long n_t,
                  const double *x, double complex *y) {
  int n_in = n_st * n_pol;
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int b = 0; b < n_beams; b++) {
    for (int s = 0; s < n_sb; s++) {
      double az = az_el[2 * b], el = az_el[2 * b + 1];
      double nb[3] = {cos(el) * sin(az), cos(el) * cos(az), sin(el)};
      double f = f0 + (double)k[s] * fs / (double)M;
      double complex *w = malloc(sizeof(double complex) * n_in);
      for (int st = 0; st < n_st; st++) {
        const double *r = enu + 3 * st;
        double proj = r[0] * nb[0] + r[1] * nb[1] + r[2] * nb[2];
        double cyc = f * proj / LPO_C;
        double fr = cyc - floor(cyc);
        double complex ph = cos(-2.0 * M_PI * fr) + I * sin(-2.0 * M_PI * fr);
        for (int p = 0; p < n_pol; p++) {
          double a = gain ? gain[st * n_pol + p] : 1.0;
          w[st * n_pol + p] = a * ph;
        }
      }
      double complex *out = y + ((long)b * n_sb + s) * n_t;
      for (long t = 0; t < n_t; t++) {
        const double *xr = x + (((long)s * n_t + t) * n_in) * 2;
        double complex acc = 0.0;
        for (int i = 0; i < n_in; i++)
          acc += w[i] * (xr[2 * i] + I * xr[2 * i + 1]);
        out[t] = acc;
      }
      free(w);
    }
  }
}

/* ---------------------------------------------------------- dedisperse */

void lpo_chirp(double f_k, double tec, int n_fft, int delay, double df,
               double complex *c) {
  double kap = lpo_kappa();
  for (int q = 0; q < n_fft; q++) {
    int qs = (q < n_fft / 2) ? q : q - n_fft;
    double nu = (double)qs * df / (double)n_fft;
    double cyc = kap * tec / (f_k + nu);
    double fr = cyc - floor(cyc);
    double cyc_d = (double)qs * (double)delay / (double)n_fft;
    double ang = -2.0 * M_PI * (fr + cyc_d);
    c[q] = cos(ang) + I * sin(ang);
  }
}

int lpo_dedisperse(int n_sb, const int *k, double f0, double fs, int M,
                   int n_tec, const double *tec, int n_fft, int hop,
                   int delay, int n_beams, long n_t, const double complex *y,
                   double complex *tail, double complex *d) {
  if (hop <= 0 || n_fft < hop || n_t % hop != 0) return -1;
  int hist = n_fft - hop;
  double df = fs / (double)M;
  long n_hop = n_t / hop;
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int b = 0; b < n_beams; b++) {
    for (int s = 0; s < n_sb; s++) {
      double f_k = f0 + (double)k[s] * df;
      const double complex *ys = y + ((long)b * n_sb + s) * n_t;
      double complex *tl = tail + ((long)b * n_sb + s) * hist;
      double complex *chirp = malloc(sizeof(double complex) * n_fft * n_tec);
      for (int j = 0; j < n_tec; j++)
        lpo_chirp(f_k, tec[j], n_fft, delay, df, chirp + (long)j * n_fft);
      double complex *U = malloc(sizeof(double complex) * n_fft);
      double complex *V = malloc(sizeof(double complex) * n_fft);
      for (long h = 0; h < n_hop; h++) {
        long start = h * hop - hist; /* stream-relative index of u[0] */
        for (int i = 0; i < n_fft; i++) {
          long t = start + i;
          U[i] = (t < 0) ? tl[hist + t] : ys[t];
        }
        lpo_fft(n_fft, U, 0);
        for (int j = 0; j < n_tec; j++) {
          const double complex *cj = chirp + (long)j * n_fft;
          for (int q = 0; q < n_fft; q++) V[q] = U[q] * cj[q];
          lpo_fft(n_fft, V, 1);
          double complex *out = d + (((long)b * n_tec + j) * n_sb + s) * n_t;
          for (int i = 0; i < hop; i++) out[h * hop + i] = V[hist + i];
        }
      }
      /* New tail: the last `hist` samples of (old tail | block). */
      double complex *nt = malloc(sizeof(double complex) * (hist > 0 ? hist : 1));
      for (int i = 0; i < hist; i++) {
        long t = n_t - hist + i;
        nt[i] = (t < 0) ? tl[hist + t] : ys[t];
      }
      memcpy(tl, nt, sizeof(double complex) * hist);
      free(nt);
      free(U);
      free(V);
      free(chirp);
    }
  }
  return 0;
}

/* ---------------------------------------------------------- synthesize */

/* Synthesis of frames [m_begin, m_end) of one series; frames m < 0 read
 * d from the history array (P-1 frames). */
static void syn_range(int M, int P, const double *h, int n_sb, const int *k,
                      long n_t, const double complex *dq,
                      const double complex *hq, long m_begin, long m_end,
                      double complex *zq) {
  double complex *ring = malloc(sizeof(double complex) * (size_t)M * P);
  double complex *X = malloc(sizeof(double complex) * M);
  for (long m = m_begin - (P - 1); m < m_end; m++) {
    /* Z_m = sum_s d_s[m] exp(+2 pi i k_s n / M): an unnormalised IDFT. */
    for (int n = 0; n < M; n++) X[n] = 0.0;
    for (int s = 0; s < n_sb; s++) {
      double complex v;
      if (m >= 0)
        v = dq[(long)s * n_t + m];
      else
        v = hq[((long)(P - 1) + m) * n_sb + s];
      X[k[s]] += v;
    }
    lpo_fft(M, X, 1);
    long slot = ((m % P) + P) % P;
    for (int n = 0; n < M; n++) ring[slot * M + n] = X[n] * (double)M;
    if (m < m_begin) continue;
    for (int n = 0; n < M; n++) {
      double complex acc = 0.0;
      for (int t = 0; t < P; t++) {
        long sl = (((m - t) % P) + P) % P;
        double g = (double)M * h[(long)t * M + n];
        acc += g * ring[sl * M + n];
      }
      zq[m * M + n] = acc;
    }
  }
  free(X);
  free(ring);
}

void lpo_synthesize(int M, int P, const double *h, int n_sb, const int *k,
                    int n_series, long n_t, const double complex *d,
                    double complex *hist, double complex *z) {
  const long chunk = 256; /* frames per parallel unit */
  long n_chunk = (n_t + chunk - 1) / chunk;
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int q = 0; q < n_series; q++) {
    for (long c = 0; c < n_chunk; c++) {
      long mb = c * chunk, me = mb + chunk < n_t ? mb + chunk : n_t;
      syn_range(M, P, h, n_sb, k, n_t, d + (long)q * n_sb * n_t,
                hist + (long)q * (P - 1) * n_sb, mb, me,
                z + (long)q * n_t * M);
    }
  }
  /* New history: the last P-1 frames of (old history | block). */
  for (int q = 0; q < n_series; q++) {
    double complex *hq = hist + (long)q * (P - 1) * n_sb;
    const double complex *dq = d + (long)q * n_sb * n_t;
    double complex *nh = malloc(sizeof(double complex) * (P - 1) * n_sb + 1);
    for (int i = 0; i < P - 1; i++) {
      long m = n_t - (P - 1) + i;
      for (int s = 0; s < n_sb; s++)
        nh[(long)i * n_sb + s] = (m >= 0) ? dq[(long)s * n_t + m]
                                          : hq[((long)(P - 1) + m) * n_sb + s];
    }
    memcpy(hq, nh, sizeof(double complex) * (P - 1) * n_sb);
    free(nh);
  }
}

/* ------------------------------------------------------ detect, trigger */

void lpo_detect(int M, long n_t, long frame0, long warm, int n_series,
                const double complex *z, double *sigma, double *wmax,
                int64_t *warg) {
#pragma omp parallel for schedule(dynamic)
  for (int q = 0; q < n_series; q++) {
    const double complex *zq = z + (long)q * n_t * M;
    double sum = 0.0;
    long cnt = 0;
    for (long m = 0; m < n_t; m++) {
      int valid = (frame0 + m) >= warm;
      double best = -1.0;
      long arg = m * M;
      for (int n = 0; n < M; n++) {
        double complex v = zq[m * M + n];
        double e = cabs(2.0 * v);
        double xr = 2.0 * creal(v);
        if (valid) {
          sum += xr * xr;
          cnt++;
        }
        if (e > best) {
          best = e;
          arg = m * M + n;
        }
      }
      wmax[(long)q * n_t + m] = best;
      warg[(long)q * n_t + m] = arg;
    }
    sigma[q] = cnt ? sqrt(sum / (double)cnt) : 0.0;
  }
}

static int trig_cmp(const void *a, const void *b) {
  const lpo_trig *x = a, *y = b;
  if (x->sample != y->sample) return x->sample < y->sample ? -1 : 1;
  return (x->tec > y->tec) - (x->tec < y->tec);
}

long lpo_trigger(int M, int P, int D, long n_t, long frame0, long warm,
                 int n_beams, int n_tec, const double *sigma,
                 const double *wmax, const int64_t *warg, double k_sigma,
                 long cap, lpo_trig *out, double *snr_peak, int *best_tec) {
  long total = 0;
  long offset = (long)M * P + (long)D * M;
  for (int b = 0; b < n_beams; b++) {
    /* Per-trial runs. */
    long n_list = 0, list_cap = 64;
    lpo_trig *list = malloc(sizeof(lpo_trig) * list_cap);
    for (int j = 0; j < n_tec; j++) {
      long q = (long)b * n_tec + j;
      double sg = sigma[q], thr = k_sigma * sg;
      const double *wm = wmax + q * n_t;
      const int64_t *wa = warg + q * n_t;
      double pk = 0.0;
      long m = 0;
      while (m < n_t) {
        int valid = (frame0 + m) >= warm;
        if (valid && sg > 0.0 && wm[m] / sg > pk) pk = wm[m] / sg;
        int fired = valid && sg > 0.0 && wm[m] > thr;
        if (!fired) {
          m++;
          continue;
        }
        long best = m;
        long e = m + 1;
        while (e < n_t && (frame0 + e) >= warm && wm[e] > thr) {
          if (wm[e] > wm[best]) best = e;
          if (wm[e] / sg > pk) pk = wm[e] / sg;
          e++;
        }
        if (n_list == list_cap) {
          list_cap *= 2;
          list = realloc(list, sizeof(lpo_trig) * list_cap);
        }
        lpo_trig t;
        t.sample = frame0 * M + wa[best] - offset;
        t.beam = b;
        t.tec = j;
        t.peak = wm[best];
        t.snr = wm[best] / sg;
        list[n_list++] = t;
        m = e;
      }
      snr_peak[q] = pk;
    }
    int bj = 0;
    for (int j = 1; j < n_tec; j++)
      if (snr_peak[(long)b * n_tec + j] > snr_peak[(long)b * n_tec + bj]) bj = j;
    best_tec[b] = bj;
    /* Cross-trial merge: chains of triggers whose consecutive samples are
     * at most M apart collapse to their best member. */
    qsort(list, n_list, sizeof(lpo_trig), trig_cmp);
    long i = 0;
    while (i < n_list) {
      long e = i + 1;
      while (e < n_list && list[e].sample - list[e - 1].sample <= M) e++;
      long best = i;
      for (long r = i + 1; r < e; r++) {
        const lpo_trig *c = &list[r], *o = &list[best];
        if (c->snr > o->snr ||
            (c->snr == o->snr &&
             (c->tec < o->tec || (c->tec == o->tec && c->sample < o->sample))))
          best = r;
      }
      if (total < cap) out[total] = list[best];
      total++;
      i = e;
    }
    free(list);
  }
  return total;
}

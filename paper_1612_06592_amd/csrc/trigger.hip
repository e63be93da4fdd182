// Trigger for the transient-buffer read-out (Winchen et al. 2016, Sec. 2).
// The paper does not define the statistic; this library triggers on the
// Hilbert envelope of the synthesised series:
//   sigma^2 = mean of (2 Re z)^2 over the block's valid samples,
//   a window (one M-sample frame) fires when its envelope maximum exceeds
//   k_sigma * sigma, each run of fired windows yields one trigger at its
//   largest maximum (earliest on ties), and per beam the triggers of all
//   trials are chained while consecutive samples are at most M apart, each
//   chain keeping its highest SNR (lowest trial, then earliest on ties).
//
// Two small kernels: per series (sigma, runs) and one merge over beams in
// beam order into the caller's list.  All reductions have a fixed
// order, so the result is bitwise reproducible.
#include <cmath>

#include "lp_internal.h"

namespace lp {

struct SynCand {
  float emax;
  int arg;
};

struct SerTrig {
  long long sample;
  float snr;
  float peak;
};

struct WorkLayout {
  int *ser_cnt;        // [ns]
  float *ser_sigma;    // [ns]
  float *ser_peak;     // [ns]
  SerTrig *ser_list;   // [ns][kTrigPerSeries]
  int *beam_cnt;       // [nb]
  lp_trig *beam_list;  // [nb][n_tec * kTrigPerSeries] rank-sorted
};

static WorkLayout layout(void *work, int n_beams, int n_tec) {
  size_t ns = (size_t)n_beams * n_tec;
  char *p = static_cast<char *>(work);
  WorkLayout w;
  w.ser_cnt = reinterpret_cast<int *>(p);
  p += ns * 4;
  w.ser_sigma = reinterpret_cast<float *>(p);
  p += ns * 4;
  w.ser_peak = reinterpret_cast<float *>(p);
  p += ns * 4;
  p += ns * 4;  // keeps the lists 16-byte aligned
  w.ser_list = reinterpret_cast<SerTrig *>(p);
  p += ns * kTrigPerSeries * sizeof(SerTrig);
  w.beam_cnt = reinterpret_cast<int *>(p);
  p += (size_t)n_beams * 16;
  w.beam_list = reinterpret_cast<lp_trig *>(p);
  return w;
}

constexpr int kT1Threads = 1024;
constexpr long kMaxTrigWindows = 1L << 20;  // fired-window bitmask in LDS

// One workgroup per series.  Pass A: coalesced reads of the window maxima;
// each wave's ballot gives the fired bits of 64 consecutive windows (LDS
// bitmask).  Pass B: each thread scans a contiguous range of the bitmask
// for run starts (a fired window whose predecessor did not fire); a
// fixed-order scan of the counts gives each run its slot.
__global__ __launch_bounds__(kT1Threads) void trig_series_kernel(
    const SynCand *__restrict__ cand, const float *__restrict__ psum,
    long n_t, long frame0, long warm, float k_sigma, long offset,
    WorkLayout w) {
  extern __shared__ unsigned bits[];          // n_t / 32 words
  __shared__ double sred[kT1Threads / 64];
  __shared__ float fred[kT1Threads / 64];
  __shared__ int ired[kT1Threads / 64];
  __shared__ int s_total;
  const int q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SynCand *cq = cand + (long)q * n_t;
  const float *pq = psum + (long)q * (n_t / 16);

  // sigma: fixed-order FP64 sum of the per-16-frame partial sums.
  const long n_part = n_t / 16;
  double acc = 0.0;
  for (long i = tid; i < n_part; i += kT1Threads) acc += (double)pq[i];
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) sred[wave] = acc;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < kT1Threads / 64; ++i) tot += sred[i];
  const long first_valid = warm > frame0 ? warm - frame0 : 0;
  const long n_valid_fr = first_valid >= n_t ? 0 : n_t - first_valid;
  const float sigma =
      n_valid_fr > 0 ? (float)sqrt(tot / ((double)n_valid_fr * kM)) : 0.0f;
  const float thr = k_sigma * sigma;
  const float inv_sigma = sigma > 0.0f ? 1.0f / sigma : 0.0f;

  // Pass A (four 64-window groups per wave and step: their loads are in
  // flight together).
  constexpr int kU = 4;
  float pk = 0.0f;
  for (long base0 = (long)wave * 64; base0 < n_t;
       base0 += (long)kT1Threads * kU) {
    float ev[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long m = base0 + (long)u * kT1Threads + lane;
      ev[u] = m < n_t ? cq[m].emax : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long base = base0 + (long)u * kT1Threads;
      if (base >= n_t) break;
      const long m = base + lane;
      const float e = ev[u];
      bool valid = m < n_t && m >= first_valid && sigma > 0.0f;
      if (valid) pk = fmaxf(pk, e / sigma);
      unsigned long long b = __ballot(valid && e > thr);
      if (lane == 0) {
        bits[base / 32] = (unsigned)b;
        if (base / 32 + 1 < (n_t + 31) / 32)
          bits[base / 32 + 1] = (unsigned)(b >> 32);
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) pk = fmaxf(pk, __shfl_xor(pk, off));
  if (lane == 0) fred[wave] = pk;
  __syncthreads();

  // Pass B.
  const long nw = (n_t + 31) / 32;
  const long per = (nw + kT1Threads - 1) / kT1Threads;
  const long w0 = (long)tid * per, w1 = min(nw, w0 + per);
  auto starts_of = [&](long wi) {
    unsigned b = bits[wi];
    unsigned prev = wi > 0 ? bits[wi - 1] >> 31 : 0u;
    return b & ~((b << 1) | prev);
  };
  int n_runs = 0;
  for (long wi = w0; wi < w1; ++wi) n_runs += __popc(starts_of(wi));
  int incl = n_runs;
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) ired[wave] = incl;
  __syncthreads();
  int wave_off = 0;
  for (int i = 0; i < wave; ++i) wave_off += ired[i];
  int pos = wave_off + incl - n_runs;
  if (tid == kT1Threads - 1) s_total = wave_off + incl;
  auto fired = [&](long m) { return (bits[m >> 5] >> (m & 31)) & 1u; };
  for (long wi = w0; wi < w1; ++wi) {
    unsigned st = starts_of(wi);
    while (st) {
      int bit = __ffs(st) - 1;
      st &= st - 1;
      long m = wi * 32 + bit;
      long best = m;
      float bv = cq[m].emax;
      for (long e = m + 1; e < n_t && fired(e); ++e) {
        float ev = cq[e].emax;
        if (ev > bv) {
          bv = ev;
          best = e;
        }
      }
      if (pos < kTrigPerSeries) {
        SerTrig t;
        t.sample = (frame0 + best) * kM + cq[best].arg - offset;
        t.peak = bv;
        t.snr = bv * inv_sigma;
        w.ser_list[(long)q * kTrigPerSeries + pos] = t;
      }
      ++pos;
    }
  }
  __syncthreads();
  if (tid == 0) {
    float p = 0.0f;
    for (int i = 0; i < kT1Threads / 64; ++i) p = fmaxf(p, fred[i]);
    w.ser_peak[q] = p;
    w.ser_sigma[q] = sigma;
    w.ser_cnt[q] = s_total;
  }
}

constexpr int kT2Threads = 256;

// One workgroup for all beams, in beam order: rank-sort each beam's
// triggers of all trials by (sample, trial), chain them, and append each
// chain's best to the caller's list (which is therefore ordered by beam,
// then sample).
__global__ __launch_bounds__(kT2Threads) void trig_merge_kernel(
    int n_beams, int n_tec, WorkLayout w, lp_trig *__restrict__ out, int cap,
    int *__restrict__ n_out, float *__restrict__ snr_out,
    int *__restrict__ best_tec, float *__restrict__ sigma_out) {
  const int tid = threadIdx.x;
  const int bcap = n_tec * kTrigPerSeries;
  __shared__ int s_n;
  int base = 0;  // meaningful in thread 0
  for (int b = 0; b < n_beams; ++b) {
    lp_trig *srt = w.beam_list + (long)b * bcap;
    if (tid == 0) {
      int o = 0;
      for (int j = 0; j < n_tec; ++j)
        o += min(w.ser_cnt[b * n_tec + j], kTrigPerSeries);
      s_n = o;
    }
    __syncthreads();
    const int N = s_n;
    for (int i = tid; i < N; i += kT2Threads) {
      int j = 0, r = i;
      while (r >= min(w.ser_cnt[b * n_tec + j], kTrigPerSeries)) {
        r -= min(w.ser_cnt[b * n_tec + j], kTrigPerSeries);
        ++j;
      }
      SerTrig ti = w.ser_list[(long)(b * n_tec + j) * kTrigPerSeries + r];
      int rank = 0;
      for (int jj = 0; jj < n_tec; ++jj) {
        int c = min(w.ser_cnt[b * n_tec + jj], kTrigPerSeries);
        const SerTrig *L = w.ser_list + (long)(b * n_tec + jj) * kTrigPerSeries;
        for (int rr = 0; rr < c; ++rr) {
          long long sj = L[rr].sample;
          if (sj < ti.sample || (sj == ti.sample && jj < j)) ++rank;
        }
      }
      lp_trig o;
      o.sample = ti.sample;
      o.beam = b;
      o.tec = j;
      o.snr = ti.snr;
      o.peak = ti.peak;
      srt[rank] = o;
    }
    __syncthreads();
    if (tid == 0) {
      int i = 0;
      while (i < N) {
        lp_trig best = srt[i];
        long long prev = best.sample;
        int e = i + 1;
        while (e < N) {
          lp_trig c = srt[e];
          if (c.sample - prev > kM) break;
          if (c.snr > best.snr ||
              (c.snr == best.snr &&
               (c.tec < best.tec ||
                (c.tec == best.tec && c.sample < best.sample))))
            best = c;
          prev = c.sample;
          ++e;
        }
        if (base < cap) out[base] = best;
        ++base;
        i = e;
      }
      int bj = 0;
      float bp = w.ser_peak[b * n_tec];
      for (int j = 0; j < n_tec; ++j) {
        float pj = w.ser_peak[b * n_tec + j];
        if (snr_out) snr_out[b * n_tec + j] = pj;
        if (sigma_out) sigma_out[b * n_tec + j] = w.ser_sigma[b * n_tec + j];
        if (pj > bp) {
          bp = pj;
          bj = j;
        }
      }
      if (best_tec) best_tec[b] = bj;
    }
    __syncthreads();
  }
  if (tid == 0) *n_out = base;
}

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_trigger(lp_ctx *ctx, const void *cand, int32_t n_beams,
                                int32_t n_tec, int64_t n_t, int64_t frame0,
                                float k_sigma, lp_trig *out, int32_t cap,
                                int32_t *n_out, float *snr_out,
                                int32_t *best_tec, float *sigma_out,
                                void *work, void *hip_stream) {
  if (!ctx || !cand || !n_out || !work || (cap > 0 && !out))
    return set_error(LP_EINVAL, "lp_trigger: NULL argument");
  if (n_beams <= 0 || n_tec <= 0 || (long)n_beams * n_tec > 65535)
    return set_error(LP_EINVAL, "lp_trigger: bad n_beams/n_tec");
  if (n_t <= 0 || n_t % kHop != 0 || n_t > kMaxTrigWindows)
    return set_error(LP_EINVAL, "lp_trigger: n_t %lld", (long long)n_t);
  if (frame0 < 0 || !(k_sigma > 0.0f) || cap < 0)
    return set_error(LP_EINVAL, "lp_trigger: bad frame0/k_sigma/cap");
  if (reinterpret_cast<uintptr_t>(work) % 16)
    return set_error(LP_EINVAL, "lp_trigger: work must be 16-byte aligned");
  lp_status rc;
  if ((rc = set_device(ctx))) return rc;
  return trig_launch(cand, n_beams, n_tec, n_t, frame0, k_sigma, out, cap,
                     n_out, snr_out, best_tec, sigma_out, work,
                     static_cast<hipStream_t>(hip_stream));
}

namespace lp {
lp_status trig_launch(const void *cand, int n_beams, int n_tec, long n_t,
                      long frame0, float k_sigma, lp_trig *out, int cap,
                      int *n_out, float *snr_out, int *best_tec,
                      float *sigma_out, void *work, hipStream_t st) {
  const int ns = n_beams * n_tec;
  WorkLayout w = layout(work, n_beams, n_tec);
  const char *cb = static_cast<const char *>(cand);
  const SynCand *cd = reinterpret_cast<const SynCand *>(cb);
  const float *ps = reinterpret_cast<const float *>(cb + (size_t)ns * n_t * 8);
  const long offset = (long)kM * kTaps + (long)kDelay * kM;
  const size_t shm = (size_t)((n_t + 31) / 32) * 4;
  LP_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(trig_series_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)shm));
  hipLaunchKernelGGL(trig_series_kernel, dim3(ns), dim3(kT1Threads), shm, st,
                     cd, ps, n_t, frame0, (long)(kDelay + kTaps), k_sigma,
                     offset, w);
  LP_HIP(hipGetLastError());
  hipLaunchKernelGGL(trig_merge_kernel, dim3(1), dim3(kT2Threads), 0, st,
                     n_beams, n_tec, w, out, cap, n_out, snr_out, best_tec,
                     sigma_out);
  LP_HIP(hipGetLastError());
  return LP_OK;
}
}  // namespace lp

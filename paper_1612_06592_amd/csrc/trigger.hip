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
// Three small kernels: per series (sigma, runs), per beam (merge), and one
// ordered compaction into the caller's list.  All reductions have a fixed
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
  lp_trig *beam_list;  // [nb][2][n_tec * kTrigPerSeries]: out | sorted
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

// One workgroup per series.
__global__ __launch_bounds__(kT1Threads) void trig_series_kernel(
    const SynCand *__restrict__ cand, const float *__restrict__ psum,
    long n_t, long frame0, long warm, float k_sigma, long offset,
    WorkLayout w) {
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

  // Each thread owns a contiguous range of windows.
  const long per = (n_t + kT1Threads - 1) / kT1Threads;
  const long w0 = (long)tid * per, w1 = min(n_t, w0 + per);
  auto fired = [&](long m) {
    return m >= first_valid && sigma > 0.0f && cq[m].emax > thr;
  };
  float pk = 0.0f;
  int n_runs = 0;
  for (long m = w0; m < w1; ++m) {
    if (m >= first_valid && sigma > 0.0f) pk = fmaxf(pk, cq[m].emax / sigma);
    if (fired(m) && !(m > 0 && fired(m - 1))) ++n_runs;
  }
  // Peak SNR: max over threads (order-free).
  for (int off = 32; off >= 1; off >>= 1) pk = fmaxf(pk, __shfl_xor(pk, off));
  // Exclusive scan of run counts (deterministic positions).
  int incl = n_runs;
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) ired[wave] = incl;
  if (lane == 0) fred[wave] = pk;
  __syncthreads();
  int wave_off = 0;
  for (int i = 0; i < wave; ++i) wave_off += ired[i];
  int pos = wave_off + incl - n_runs;
  if (tid == kT1Threads - 1) s_total = wave_off + incl;
  for (long m = w0; m < w1; ++m) {
    if (!(fired(m) && !(m > 0 && fired(m - 1)))) continue;
    long best = m;
    for (long e = m + 1; e < n_t && fired(e); ++e)
      if (cq[e].emax > cq[best].emax) best = e;
    if (pos < kTrigPerSeries) {
      SerTrig t;
      t.sample = (frame0 + best) * kM + cq[best].arg - offset;
      t.peak = cq[best].emax;
      t.snr = cq[best].emax / sigma;
      w.ser_list[(long)q * kTrigPerSeries + pos] = t;
    }
    ++pos;
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

// One workgroup per beam: rank-sort the trials' triggers by (sample,
// trial), then chain and keep each chain's best.
__global__ __launch_bounds__(kT2Threads) void trig_beam_kernel(
    int n_tec, WorkLayout w, float *__restrict__ snr_out,
    int *__restrict__ best_tec, float *__restrict__ sigma_out) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int cap = n_tec * kTrigPerSeries;
  lp_trig *bl = w.beam_list + (long)b * 2 * cap;  // chain representatives
  lp_trig *srt = bl + cap;                        // rank-sorted triggers
  __shared__ int s_off[65];
  if (tid == 0) {
    int o = 0;
    for (int j = 0; j < n_tec; ++j) {
      int c = min(w.ser_cnt[b * n_tec + j], kTrigPerSeries);
      o += c;
    }
    s_off[0] = o;
  }
  __syncthreads();
  const int N = s_off[0];
  // Ranks are unique, so each trigger lands in its own sorted slot.
  for (int i = tid; i < N; i += kT2Threads) {
    // Locate element i: walk trials.
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
    // Walk the sorted list and keep one representative per chain.
    int out = 0;
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
             (c.tec < best.tec || (c.tec == best.tec && c.sample < best.sample))))
          best = c;
        prev = c.sample;
        ++e;
      }
      bl[out++] = best;
      i = e;
    }
    w.beam_cnt[b] = out;
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
}

// Ordered compaction of the per-beam lists into the caller's array.
__global__ __launch_bounds__(256) void trig_compact_kernel(
    int n_beams, int n_tec, WorkLayout w, lp_trig *__restrict__ out, int cap,
    int *__restrict__ n_out) {
  __shared__ int s_base;
  const int stride = 2 * n_tec * kTrigPerSeries;
  int base = 0;
  for (int b = 0; b < n_beams; ++b) {
    int c = w.beam_cnt[b];
    for (int i = threadIdx.x; i < c; i += blockDim.x)
      if (base + i < cap) out[base + i] = w.beam_list[(long)b * stride + i];
    base += c;
  }
  if (threadIdx.x == 0) {
    s_base = base;
    *n_out = s_base;
  }
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
  if (n_t <= 0 || n_t % kHop != 0)
    return set_error(LP_EINVAL, "lp_trigger: n_t %lld", (long long)n_t);
  if (frame0 < 0 || !(k_sigma > 0.0f) || cap < 0)
    return set_error(LP_EINVAL, "lp_trigger: bad frame0/k_sigma/cap");
  if (reinterpret_cast<uintptr_t>(work) % 16)
    return set_error(LP_EINVAL, "lp_trigger: work must be 16-byte aligned");
  lp_status rc;
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int ns = n_beams * n_tec;
  WorkLayout w = layout(work, n_beams, n_tec);
  const char *cb = static_cast<const char *>(cand);
  const SynCand *cd = reinterpret_cast<const SynCand *>(cb);
  const float *ps = reinterpret_cast<const float *>(cb + (size_t)ns * n_t * 8);
  const long offset = (long)kM * kTaps + (long)kDelay * kM;
  hipLaunchKernelGGL(trig_series_kernel, dim3(ns), dim3(kT1Threads), 0, st,
                     cd, ps, (long)n_t, (long)frame0, (long)(kDelay + kTaps),
                     k_sigma, offset, w);
  LP_HIP(hipGetLastError());
  hipLaunchKernelGGL(trig_beam_kernel, dim3(n_beams), dim3(kT2Threads), 0, st,
                     n_tec, w, snr_out, best_tec, sigma_out);
  LP_HIP(hipGetLastError());
  hipLaunchKernelGGL(trig_compact_kernel, dim3(1), dim3(256), 0, st, n_beams,
                     n_tec, w, out, cap, n_out);
  LP_HIP(hipGetLastError());
  return LP_OK;
}

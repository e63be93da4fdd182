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
// Four kernels, every list exact (a series of n_t windows has at most n_t/2
// runs, and the workspace holds that many):
//   trig_series_kernel  one workgroup per series: sigma, fired-window
//                       bitmask in LDS, every run's maximum in time order;
//   trig_merge_kernel   one workgroup per beam: the rank of each trigger in
//                       the beam's (sample, trial) order by binary searches
//                       in the other trials' sorted lists, then the chains
//                       by a segmented scan over the sorted sequence;
//   trig_scan_kernel    one workgroup: each beam's first output slot, the
//                       true total, per-series SNR / sigma, best trial;
//   trig_copy_kernel    one workgroup per beam: its chains into the list.
// All reductions have a fixed order, so the result is bitwise reproducible.
#include <cmath>

#include "lp_internal.h"

namespace lp {

struct SynCand {
  float emax;
  int arg;
};

// One run's trigger: pos = frame * M + offset in the frame (block-relative),
// peak = the envelope there.
struct SerEnt {
  int pos;
  float peak;
};

struct WorkLayout {
  int *ser_cnt;      // [ns] runs per series
  float *ser_sigma;  // [ns]
  float *ser_peak;   // [ns] largest envelope / sigma over valid windows
  float *ser_inv;    // [ns] 1 / sigma in FP32 (0 when sigma is 0)
  int *beam_cnt;     // [nb] chains per beam
  int *beam_base;    // [nb] first output slot of each beam
  SerEnt *ser_list;  // [ns][cap_s] in time order
  unsigned *sorted;  // [nb][n_tec * cap_s] (trial << 20 | index), merged order
  unsigned *chains;  // [nb][n_tec * cap_s] best member of each chain
  long cap_s;        // n_t / 2
};

static size_t al16(size_t n) { return (n + 15) & ~(size_t)15; }

static size_t work_bytes(long n_beams, long n_tec, long n_t) {
  const size_t ns = (size_t)n_beams * n_tec, cap_s = (size_t)n_t / 2;
  return al16(ns * 16 + (size_t)n_beams * 8) + ns * cap_s * sizeof(SerEnt) +
         2 * ns * cap_s * sizeof(unsigned);
}

static WorkLayout layout(void *work, int n_beams, int n_tec, long n_t) {
  const size_t ns = (size_t)n_beams * n_tec, cap_s = (size_t)n_t / 2;
  char *p = static_cast<char *>(work);
  WorkLayout w;
  w.ser_cnt = reinterpret_cast<int *>(p);
  w.ser_sigma = reinterpret_cast<float *>(p + ns * 4);
  w.ser_peak = reinterpret_cast<float *>(p + ns * 8);
  w.ser_inv = reinterpret_cast<float *>(p + ns * 12);
  w.beam_cnt = reinterpret_cast<int *>(p + ns * 16);
  w.beam_base = reinterpret_cast<int *>(p + ns * 16 + (size_t)n_beams * 4);
  p += al16(ns * 16 + (size_t)n_beams * 8);
  w.ser_list = reinterpret_cast<SerEnt *>(p);
  p += ns * cap_s * sizeof(SerEnt);
  w.sorted = reinterpret_cast<unsigned *>(p);
  p += ns * cap_s * sizeof(unsigned);
  w.chains = reinterpret_cast<unsigned *>(p);
  w.cap_s = (long)cap_s;
  return w;
}

constexpr int kT1Threads = 1024;
constexpr long kMaxTrigWindows = 1L << 20;  // fired-window bitmask in LDS
constexpr int kIdxBits = 20;                // index bits of a packed entry

// Workgroup-wide exclusive scan of one int per thread (1024 threads);
// returns the exclusive prefix and sets *total.  `scratch` holds 16 ints.
__device__ __forceinline__ int wg_exscan(int v, int *scratch, int *total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  __syncthreads();  // scratch free from any previous use
  if (lane == 63) scratch[wave] = incl;
  __syncthreads();
  int wave_off = 0, tot = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    const int s = scratch[i];
    if (i < wave) wave_off += s;
    tot += s;
  }
  *total = tot;
  return wave_off + incl - v;
}

// One workgroup per series.  Pass A: coalesced reads of the window maxima;
// each wave's ballot gives the fired bits of 64 consecutive windows (LDS
// bitmask).  Pass B: each thread scans a contiguous range of the bitmask
// for run starts (a fired window whose predecessor did not fire); a
// fixed-order scan of the counts gives each run its slot in the series'
// list, so the list is in time order.
__global__ __launch_bounds__(kT1Threads) void trig_series_kernel(
    const SynCand *__restrict__ cand, const float *__restrict__ psum,
    long n_t, long frame0, long warm, float k_sigma, WorkLayout w) {
  extern __shared__ unsigned bits[];          // n_t / 32 words
  __shared__ double sred[kT1Threads / 64];
  __shared__ float fred[kT1Threads / 64];
  __shared__ int ired[kT1Threads / 64];
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
  int total = 0;
  int pos = wg_exscan(n_runs, ired, &total);
  auto fired = [&](long m) { return (bits[m >> 5] >> (m & 31)) & 1u; };
  SerEnt *list = w.ser_list + (long)q * w.cap_s;
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
      SerEnt t;
      t.pos = (int)(best * kM) + cq[best].arg;
      t.peak = bv;
      list[pos++] = t;  // pos < n_t / 2: runs are separated by a gap
    }
  }
  if (tid == 0) {
    float p = 0.0f;
    for (int i = 0; i < kT1Threads / 64; ++i) p = fmaxf(p, fred[i]);
    w.ser_peak[q] = p;
    w.ser_sigma[q] = sigma;
    w.ser_inv[q] = inv_sigma;
    w.ser_cnt[q] = total;
  }
}

constexpr int kT2Threads = 1024;

// A candidate chain best: SNR, trial, block position, packed entry.
struct Best {
  float snr;
  int tec;
  int pos;
  unsigned u;  // 0xffffffff: none
};

__device__ __forceinline__ bool better(const Best &c, const Best &o) {
  if (o.u == 0xffffffffu) return c.u != 0xffffffffu;
  if (c.u == 0xffffffffu) return false;
  return c.snr > o.snr ||
         (c.snr == o.snr &&
          (c.tec < o.tec || (c.tec == o.tec && c.pos < o.pos)));
}

__device__ __forceinline__ Best best_of(const Best &a, const Best &b) {
  return better(b, a) ? b : a;
}

__device__ __forceinline__ Best shfl_up_best(const Best &v, int off) {
  Best r;
  r.snr = __shfl_up(v.snr, off);
  r.tec = __shfl_up(v.tec, off);
  r.pos = __shfl_up(v.pos, off);
  r.u = (unsigned)__shfl_up((int)v.u, off);
  return r;
}

// First index in the ascending list L[0..n) whose pos is > s (UPPER) or
// >= s (lower).
template <bool UPPER>
__device__ __forceinline__ int search(const SerEnt *__restrict__ L, int n,
                                      int s) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int p = L[mid].pos;
    if (UPPER ? (p <= s) : (p < s))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One workgroup per beam.  Phase 1: every trigger of every trial of the
// beam gets its rank in (sample, trial) order -- its index in its own
// trial's time-ordered list plus, for every other trial, the number of
// entries before it (binary search) -- and is written to that rank.
// Phase 2: thread t takes a contiguous range of the merged sequence; a
// chain starts where the sample advances by more than M.  Each range's
// start count, the best of its head (before its first start) and of its
// tail (from its last start) go through a workgroup scan -- an exclusive
// sum of starts for the chain ids, and a segmented maximum that carries
// the best of the open chain from range to range -- and each chain's best
// is written once, by the thread in whose range the chain ends.
__global__ __launch_bounds__(kT2Threads) void trig_merge_kernel(int n_tec,
                                                                WorkLayout w) {
  extern __shared__ int off[];  // [n_tec + 1] first merged slot per trial
  __shared__ int iscr[kT2Threads / 64];
  __shared__ Best bscr[kT2Threads / 64];
  __shared__ int fscr[kT2Threads / 64];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long s0 = (long)b * n_tec;
  const int *cnt = w.ser_cnt + s0;
  const SerEnt *lists = w.ser_list + s0 * w.cap_s;
  unsigned *srt = w.sorted + s0 * w.cap_s;
  unsigned *chn = w.chains + s0 * w.cap_s;

  // Offsets of the trials' lists in the merged sequence.
  int carry = 0;
  for (int j0 = 0; j0 < n_tec; j0 += kT2Threads) {
    const int j = j0 + tid;
    const int c = j < n_tec ? cnt[j] : 0;
    int tot = 0;
    const int ex = wg_exscan(c, iscr, &tot);
    if (j < n_tec) off[j] = carry + ex;
    carry += tot;
  }
  if (tid == 0) off[n_tec] = carry;
  __syncthreads();
  const int N = carry;

  // Phase 1: ranks.
  for (int e = tid; e < N; e += kT2Threads) {
    int lo = 0, hi = n_tec;  // largest j with off[j] <= e
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= e)
        lo = mid;
      else
        hi = mid;
    }
    const int j = lo, i = e - off[j];
    const int s = lists[(long)j * w.cap_s + i].pos;
    int rank = i;
    for (int jj = 0; jj < n_tec; ++jj) {
      if (jj == j) continue;
      const int c = off[jj + 1] - off[jj];
      if (c == 0) continue;
      const SerEnt *L = lists + (long)jj * w.cap_s;
      rank += jj < j ? search<true>(L, c, s) : search<false>(L, c, s);
    }
    srt[rank] = ((unsigned)j << kIdxBits) | (unsigned)i;
  }
  __syncthreads();

  // Phase 2: chains.
  auto entry = [&](int r) {
    const unsigned u = srt[r];
    const int j = (int)(u >> kIdxBits), i = (int)(u & ((1u << kIdxBits) - 1));
    const SerEnt e = lists[(long)j * w.cap_s + i];
    Best v;
    v.snr = e.peak * w.ser_inv[s0 + j];
    v.tec = j;
    v.pos = e.pos;
    v.u = u;
    return v;
  };
  const Best none = {0.0f, 0, 0, 0xffffffffu};
  const int per = (N + kT2Threads - 1) / kT2Threads;
  const int r0 = (int)min((long)N, (long)tid * per);
  const int r1 = (int)min((long)N, (long)r0 + per);
  int n_starts = 0;
  Best head = none, tail = none;
  int prev = r0 > 0 ? entry(r0 - 1).pos : 0;
  for (int r = r0; r < r1; ++r) {
    const Best v = entry(r);
    const bool start = r == 0 || v.pos - prev > kM;
    prev = v.pos;
    if (start) {
      ++n_starts;
      tail = v;
    } else if (n_starts == 0) {
      head = best_of(head, v);
    } else {
      tail = best_of(tail, v);
    }
  }
  int n_chains = 0;
  const int cid0 = wg_exscan(n_starts, iscr, &n_chains);
  // Segmented inclusive scan over threads of (has start, open-chain best):
  // S_t = best of the chain still open at the end of range t.
  const int flag = n_starts > 0;
  Best val = flag ? tail : head;
  int f = flag;
  for (int o = 1; o < 64; o <<= 1) {
    const Best pv = shfl_up_best(val, o);
    const int pf = __shfl_up(f, o);
    if (lane >= o) {
      if (!f) val = best_of(pv, val);
      f |= pf;
    }
  }
  if (lane == 63) {
    bscr[wave] = val;
    fscr[wave] = f;
  }
  __syncthreads();
  // Carry into this wave: the segmented scan of the earlier waves' totals.
  Best cin = none;
  for (int i = 0; i < wave; ++i) {
    cin = fscr[i] ? bscr[i] : best_of(cin, bscr[i]);
  }
  if (!f) val = best_of(cin, val);
  // S_{t-1}: the open-chain best before this range.
  Best before = shfl_up_best(val, 1);
  if (lane == 0) before = cin;
  if (flag && cid0 > 0) {
    // The chain open before this range ends at its first start.
    chn[cid0 - 1] = best_of(before, head).u;
  }
  if (flag) {
    // Chains that start and end inside this range.
    int k = 0;
    Best cur = none;
    int pp = r0 > 0 ? entry(r0 - 1).pos : 0;
    for (int r = r0; r < r1; ++r) {
      const Best v = entry(r);
      const bool start = r == 0 || v.pos - pp > kM;
      pp = v.pos;
      if (start) {
        if (k > 0) chn[cid0 + k - 1] = cur.u;
        ++k;
        cur = v;
      } else if (k > 0) {
        cur = best_of(cur, v);
      }
    }
  }
  // The last chain ends at the end of the sequence.
  if (N > 0 && r0 < N && r1 == N) chn[n_chains - 1] = val.u;
  if (tid == 0) w.beam_cnt[b] = n_chains;
}

// One workgroup: each beam's first slot, the true total, per-series SNR and
// sigma, best trial per beam (lowest on ties).
__global__ __launch_bounds__(kT2Threads) void trig_scan_kernel(
    int n_beams, int n_tec, WorkLayout w, int *__restrict__ n_out,
    float *__restrict__ snr_out, int *__restrict__ best_tec,
    float *__restrict__ sigma_out) {
  __shared__ int iscr[kT2Threads / 64];
  const int tid = threadIdx.x;
  int carry = 0;
  for (int b0 = 0; b0 < n_beams; b0 += kT2Threads) {
    const int b = b0 + tid;
    const int c = b < n_beams ? w.beam_cnt[b] : 0;
    int tot = 0;
    const int ex = wg_exscan(c, iscr, &tot);
    if (b < n_beams) w.beam_base[b] = carry + ex;
    carry += tot;
  }
  if (tid == 0) *n_out = carry;
  const long ns = (long)n_beams * n_tec;
  for (long q = tid; q < ns; q += kT2Threads) {
    if (snr_out) snr_out[q] = w.ser_peak[q];
    if (sigma_out) sigma_out[q] = w.ser_sigma[q];
  }
  if (best_tec) {
    for (int b = tid; b < n_beams; b += kT2Threads) {
      const float *pk = w.ser_peak + (long)b * n_tec;
      int bj = 0;
      float bp = pk[0];
      for (int j = 1; j < n_tec; ++j)
        if (pk[j] > bp) {
          bp = pk[j];
          bj = j;
        }
      best_tec[b] = bj;
    }
  }
}

// One workgroup per beam: its chains, in sample order, into out[base ..]
// (slots at or past cap are dropped; n_out keeps the true count).
__global__ __launch_bounds__(256) void trig_copy_kernel(
    int n_tec, long frame0, long offset, WorkLayout w,
    lp_trig *__restrict__ out, int cap) {
  const int b = blockIdx.x;
  const long s0 = (long)b * n_tec;
  const int n = w.beam_cnt[b], base = w.beam_base[b];
  const unsigned *chn = w.chains + s0 * w.cap_s;
  const SerEnt *lists = w.ser_list + s0 * w.cap_s;
  for (int c = threadIdx.x; c < n && base + c < cap; c += 256) {
    const unsigned u = chn[c];
    const int j = (int)(u >> kIdxBits), i = (int)(u & ((1u << kIdxBits) - 1));
    const SerEnt e = lists[(long)j * w.cap_s + i];
    lp_trig t;
    t.sample = frame0 * kM - offset + e.pos;
    t.beam = b;
    t.tec = j;
    t.snr = e.peak * w.ser_inv[s0 + j];
    t.peak = e.peak;
    out[base + c] = t;
  }
}

}  // namespace lp

using namespace lp;

extern "C" size_t lp_trigger_work_bytes(int32_t n_beams, int32_t n_tec,
                                        int64_t n_t) {
  if (n_beams <= 0 || n_tec <= 0 || n_t <= 0) return 0;
  return work_bytes(n_beams, n_tec, n_t);
}

namespace lp {
lp_status check_trigger_args(int n_beams, int n_tec, long n_t, long frame0,
                             float k_sigma, int cap) {
  if (n_beams <= 0 || n_tec <= 0 || (long)n_beams * n_tec > 65535 ||
      n_tec > 4096)
    return set_error(LP_EINVAL, "lp_trigger: bad n_beams %d / n_tec %d",
                     n_beams, n_tec);
  if (n_t <= 0 || n_t % kHop != 0 || n_t > kMaxTrigWindows)
    return set_error(LP_EINVAL, "lp_trigger: n_t %lld", (long long)n_t);
  // Packed merged entries and per-beam ranks are 32-bit: a beam's trials
  // hold at most n_tec * n_t / 2 triggers, below 2^31.
  if ((long)n_tec * (n_t / 2) >= (1L << 31) ||
      (long)n_beams * n_tec * (n_t / 2) >= (1L << 31))
    return set_error(LP_EINVAL, "lp_trigger: n_beams * n_tec * n_t too large");
  if (frame0 < 0 || !(k_sigma > 0.0f) || cap < 0)
    return set_error(LP_EINVAL, "lp_trigger: bad frame0/k_sigma/cap");
  return LP_OK;
}
}  // namespace lp

extern "C" lp_status lp_trigger(lp_ctx *ctx, const void *cand, int32_t n_beams,
                                int32_t n_tec, int64_t n_t, int64_t frame0,
                                float k_sigma, lp_trig *out, int32_t cap,
                                int32_t *n_out, float *snr_out,
                                int32_t *best_tec, float *sigma_out,
                                void *work, void *hip_stream) {
  if (!ctx || !cand || !n_out || !work || (cap > 0 && !out))
    return set_error(LP_EINVAL, "lp_trigger: NULL argument");
  lp_status rc = check_trigger_args(n_beams, n_tec, n_t, frame0, k_sigma, cap);
  if (rc) return rc;
  if (reinterpret_cast<uintptr_t>(work) % 16)
    return set_error(LP_EINVAL, "lp_trigger: work must be 16-byte aligned");
  if ((rc = set_device(ctx))) return rc;
  return trig_launch(cand, n_beams, n_tec, n_t, frame0, k_sigma, out, cap,
                     n_out, snr_out, best_tec, sigma_out, work,
                     static_cast<hipStream_t>(hip_stream));
}

// ---- lp_trigger_noalloc: the workspace in a fixed device array ----------
// One copy per device, LP_TRIGGER_SCRATCH_BYTES long, held until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host the
// name is only a stand-in): lp_ctx_create takes its device address once per
// device with hipGetSymbolAddress, and every launch uses that address.
static __device__ __align__(256) unsigned char scratch[LP_TRIGGER_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

namespace lp {
// Called by lp_ctx_create with `device` current.
lp_status trig_scratch_attach(int device) {
  if (device < 0 || device >= kMaxScratchDevices)
    return set_error(LP_EINVAL, "device %d beyond the scratch table", device);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return LP_OK;
  void *ptr = nullptr;
  LP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256)
    return set_error(LP_EHIP, "trigger scratch: bad device address %p", ptr);
  g_scratch_ptr[device] = ptr;
  return LP_OK;
}
}  // namespace lp

extern "C" lp_status lp_trigger_noalloc(lp_ctx *ctx, const void *cand,
                                        int32_t n_beams, int32_t n_tec,
                                        int64_t n_t, int64_t frame0,
                                        float k_sigma, lp_trig *out,
                                        int32_t cap, int32_t *n_out,
                                        float *snr_out, int32_t *best_tec,
                                        float *sigma_out, void *hip_stream) {
  if (!ctx || !cand || !n_out || (cap > 0 && !out))
    return set_error(LP_EINVAL, "lp_trigger_noalloc: NULL argument");
  lp_status rc = check_trigger_args(n_beams, n_tec, n_t, frame0, k_sigma, cap);
  if (rc) return rc;
  const size_t need = work_bytes(n_beams, n_tec, n_t);
  if (need > LP_TRIGGER_SCRATCH_BYTES)
    return set_error(LP_EINVAL,
                     "lp_trigger_noalloc: %d beams x %d trials x %lld samples "
                     "need %zu bytes of workspace, above the fixed %zu",
                     n_beams, n_tec, (long long)n_t, need,
                     (size_t)LP_TRIGGER_SCRATCH_BYTES);
  if ((rc = set_device(ctx))) return rc;
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxScratchDevices)
      ptr = g_scratch_ptr[ctx->device];
  }
  if (!ptr)
    return set_error(LP_EHIP, "lp_trigger_noalloc: no scratch address for "
                              "device %d", ctx->device);
  // Every workspace word the kernels read is written earlier in the same
  // call, so nothing needs clearing between calls.
  return trig_launch(cand, n_beams, n_tec, n_t, frame0, k_sigma, out, cap,
                     n_out, snr_out, best_tec, sigma_out, ptr,
                     static_cast<hipStream_t>(hip_stream));
}

namespace lp {
lp_status trig_launch(const void *cand, int n_beams, int n_tec, long n_t,
                      long frame0, float k_sigma, lp_trig *out, int cap,
                      int *n_out, float *snr_out, int *best_tec,
                      float *sigma_out, void *work, hipStream_t st) {
  const int ns = n_beams * n_tec;
  WorkLayout w = layout(work, n_beams, n_tec, n_t);
  const char *cb = static_cast<const char *>(cand);
  const SynCand *cd = reinterpret_cast<const SynCand *>(cb);
  const float *ps = reinterpret_cast<const float *>(cb + (size_t)ns * n_t * 8);
  const long offset = (long)kM * kTaps + (long)kDelay * kM;
  const size_t shm = (size_t)((n_t + 31) / 32) * 4;
  LP_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(trig_series_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)shm));
  hipLaunchKernelGGL(trig_series_kernel, dim3(ns), dim3(kT1Threads), shm, st,
                     cd, ps, n_t, frame0, (long)(kDelay + kTaps), k_sigma, w);
  LP_HIP(hipGetLastError());
  hipLaunchKernelGGL(trig_merge_kernel, dim3(n_beams), dim3(kT2Threads),
                     (size_t)(n_tec + 1) * 4, st, n_tec, w);
  LP_HIP(hipGetLastError());
  hipLaunchKernelGGL(trig_scan_kernel, dim3(1), dim3(kT2Threads), 0, st,
                     n_beams, n_tec, w, n_out, snr_out, best_tec, sigma_out);
  LP_HIP(hipGetLastError());
  hipLaunchKernelGGL(trig_copy_kernel, dim3(n_beams), dim3(256), 0, st, n_tec,
                     frame0, offset, w, out, cap);
  LP_HIP(hipGetLastError());
  return LP_OK;
}
}  // namespace lp

// Internal declarations of liblp.so (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lp.h"

namespace lp {

constexpr double kC = 299792458.0;  // speed of light, m/s
constexpr int kM = LP_M;
constexpr int kTaps = LP_TAPS;
constexpr int kNfft = LP_NFFT;
constexpr int kHop = LP_HOP;
constexpr int kDelay = LP_DELAY;
constexpr int kHist = kNfft - kHop;   // overlap-save history per series
constexpr int kSynHist = 16;          // synthesis history frames kept

// Thread-local error reporting.
lp_status set_error(lp_status code, const char *fmt, ...);
lp_status hip_fail(hipError_t e, const char *what);

#define LP_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return lp::hip_fail(e_, #call); \
  } while (0)

// First-fit allocator over [0, size) (256-byte granules): the serving
// arena and the context's bound constant buffer.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  static size_t round(size_t n) { return (std::max<size_t>(n, 1) + 255) & ~(size_t)255; }
  void init(size_t n) {
    size = n;
    free_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t *off) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        size_t rest = it->second - n, pos = it->first + n;
        free_.erase(it);
        if (rest) free_[pos] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t t = 0;
    for (auto &kv : free_) t += kv.second;
    return t;
  }
};

// Device memory of a plan table: from the context's bound constant buffer
// (arena != NULL) or from hipMalloc.
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  Arena *arena = nullptr;
  size_t off = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (!p) return;
    if (arena)
      arena->release(off, n);
    else
      (void)hipFree(p);
    p = nullptr;
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
};

// A cached table set.  `refs` counts holders: entry points during a call
// and open serving streams; only plans nobody holds are evicted.  Tables
// are written by kernels and copies on the stream of the call that made
// the plan; `ready` is recorded there, and a launch on another stream
// waits for it once.
struct PlanBase {
  std::vector<uint8_t> key;  // first byte: kind
  int refs = 0;
  uint64_t tick = 0;         // last lookup (LRU)
  size_t bytes = 0;          // device bytes of the tables
  hipEvent_t ready = nullptr;
  hipStream_t made_on = nullptr;
  std::atomic<bool> ready_seen{false};
  std::vector<std::vector<uint8_t>> host;  // sources of the async uploads
  virtual ~PlanBase() {
    if (ready) (void)hipEventDestroy(ready);
  }
};

// Beam-weight table for one (array, band, beam set, precision, sample type).
struct BfPlan : PlanBase {
  int prec = 0;
  int n_in = 0, n_beams = 0, n_sb = 0;
  int KS = 0, NT = 0;        // MFMA: k-steps of 16 real rows, n-tiles of 16
  bool scaled = false;       // per-input power-of-two input scaling in use
  DevBuf params;             // descriptor copies the weight kernel reads
  DevBuf w;                  // FP16 MFMA fragments or FP32 [s][in][b]
  DevBuf xscale;             // FP16 [KS*16] input scale factors (MFMA)
};

// Chirp constants for one (band, TEC list).
struct DdPlan : PlanBase {
  int n_tec = 0, n_sb = 0;
  DevBuf params;  // f64 [J] TEC, i32 [S] subband ids
  DevBuf base;    // f32 [J][S] frac(kappa T / f_k) in cycles
  DevBuf afac;    // f32 [J][S] kappa T / f_k in cycles
  DevBuf rfk;     // f32 [S] (subband rate / N_fft) / f_k
  DevBuf gq;      // f32 [S][N_fft] x / (1 + x), x = nu_q / f_k (signed bin q)
  // float2 [S][N_fft] factor from one trial's chirp to the next's on a
  // uniform grid (present when `uniform`).
  DevBuf rstep;
  bool uniform = false;  // n_tec >= 2 trials spaced by a constant dT
};

// Synthesis tables for one (band, prototype beta).
struct SynPlan : PlanBase {
  DevBuf taps;    // f32 [16][1024] g = M h
  DevBuf taps2;   // f32 [16][1024] 2 g (synthesis of 2 z)
  DevBuf binmap;  // i16 [512] subband position of bin k, or -1
  DevBuf kbin;    // i16 [n_sb] bin k of each subband position
  int kmax = 511;  // highest bin of the band
};

// Two-stage beamforming: stage-2 coefficients for one (array, grouping,
// band, preliminary and final directions).
struct TsPlan : PlanBase {
  int G = 0, P = 0, B = 0, S = 0;
  DevBuf coef;    // float2 [S][B][G]
  DevBuf order;   // i32 [B] final beams ordered by their preliminary beam
  DevBuf pstart;  // i32 [P + 1] ranges of `order` per preliminary beam
};

enum PlanKind : uint8_t { kPlanBf = 1, kPlanDd, kPlanSyn, kPlanTs };

}  // namespace lp

struct lp_ctx {
  int device = 0;
  int n_cu = 256;     // compute units of the device
  lp::DevBuf tw4096;  // float2 exp(-2 pi i n / 4096), n < 4096
  std::mutex mu;      // guards everything below
  uint64_t tick = 0;
  size_t plan_max = 64;          // cached plans kept beyond those held
  bool bound = false;            // plan tables come from the caller's buffer
  char *const_base = nullptr;
  lp::Arena const_arena;
  std::vector<std::unique_ptr<lp::PlanBase>> plans;  // destroyed first
};

namespace lp {

// Word 3 of a raw (untyped, stride 0) buffer resource on CDNA: 32-bit data
// format, so bounds-checked dword loads are valid (offsets past the
// resource's size read as zero).
constexpr int kRawBufferWord3 = 0x00020000;

// Beamformer input shapes every launch supports: at most 128 inputs, a
// time row (n_in complex samples) a multiple of 4 bytes, and on the
// FP16-MFMA path a row of at most 256 bytes (the kernel's staging tile).
// Returns NULL when supported, else the reason.
inline const char *bf_shape_error(int n_in, int dtype, int prec) {
  if (n_in <= 0 || n_in > 128) return "n_st * n_pol must be in 1..128";
  const int row = 2 * n_in * (dtype == LP_CI8 ? 1 : 2);
  if (row % 4 != 0) return "a time row must be a multiple of 4 bytes";
  if (prec == LP_FP16_MFMA && row > 256)
    return "FP16-MFMA needs time rows of at most 256 bytes "
           "(int16 samples: at most 64 inputs)";
  return nullptr;
}

// Plan cache (ctx.hip).  A lookup returns the plan held (refs + 1); the
// holder releases it.  A new plan's tables are written asynchronously on
// the caller's stream.
template <class T>
struct PlanRef {
  lp_ctx *ctx = nullptr;
  T *p = nullptr;
  PlanRef() = default;
  PlanRef(const PlanRef &) = delete;
  PlanRef &operator=(const PlanRef &) = delete;
  ~PlanRef();
  T *operator->() const { return p; }
  T *get() const { return p; }
  T *keep() {  // the caller now owns the hold (serving streams)
    T *q = p;
    p = nullptr;
    return q;
  }
};
void plan_release(lp_ctx *ctx, PlanBase *p);
template <class T>
PlanRef<T>::~PlanRef() {
  if (p) plan_release(ctx, p);
}
// Under ctx->mu: the cached plan with this key (held), or NULL.
PlanBase *plan_find(lp_ctx *ctx, const std::vector<uint8_t> &key);
// Under ctx->mu: device memory for a table of a plan being made.
lp_status plan_alloc(lp_ctx *ctx, PlanBase *p, DevBuf &b, size_t n);
// Under ctx->mu: copy host bytes (kept in the plan) to a table on st.
lp_status plan_upload(PlanBase *p, DevBuf &b, const void *src, size_t n,
                      hipStream_t st);
// Under ctx->mu: record readiness on st, cache the plan (held) and evict
// unheld plans beyond the cache size.
lp_status plan_insert(lp_ctx *ctx, std::unique_ptr<PlanBase> p,
                      hipStream_t st);
// Before launching with a plan on st: order st after the plan's tables.
lp_status plan_wait(PlanBase *p, hipStream_t st);

lp_status get_bf_plan(lp_ctx *ctx, const lp_array *a, const lp_band *band,
                      const lp_dir *beams, int n_beams, int prec, int dtype,
                      hipStream_t st, PlanRef<BfPlan> &out,
                      const int *st_group = nullptr,
                      const int *beam_group = nullptr);
lp_status get_dd_plan(lp_ctx *ctx, const lp_band *band, const double *tec,
                      int n_tec, hipStream_t st, PlanRef<DdPlan> &out);
lp_status get_syn_plan(lp_ctx *ctx, const lp_band *band, hipStream_t st,
                       PlanRef<SynPlan> &out);
lp_status check_band(const lp_band *band);
lp_status set_device(lp_ctx *ctx);
// Takes the device address of lp_trigger_noalloc's fixed workspace for
// `device` (current); once per device, later calls return at once.
lp_status trig_scratch_attach(int device);

// Stage launches on an explicit stream, without argument checks (the
// public entry points and the serving loop validate first).
//   x rows of subband s start at x + (s * x_nt + x_t0) * 2 * n_in samples;
//   cand rows are cand_nt frames long and the block starts at cand_t0.
lp_status bf_launch(BfPlan *p, const void *x, int dtype, long x_nt,
                    long x_t0, long n_t, int n_sb, void *y, hipStream_t st);
//   dd_launch runs trials j0 .. j0 + nj - 1 of the plan's list (d holds nj
//   trials per beam); syn_launch fills series series0 .. series0 + n_series
//   - 1 of a candidate array laid out for n_series_total series.
lp_status dd_launch(lp_ctx *ctx, DdPlan *p, int n_sb, const void *y,
                    int n_beams, long n_t, void *tail, bool update_tail,
                    void *d, int j0, int nj, hipStream_t st);
lp_status syn_launch(lp_ctx *ctx, SynPlan *p, int n_sb, const void *d,
                     int n_series, long n_t, long frame0, void *hist,
                     float *x_out, void *cand, long cand_nt, long cand_t0,
                     int series0, int n_series_total, hipStream_t st);
// Argument checks shared by lp_trigger and the serving loop.
lp_status check_trigger_args(int n_beams, int n_tec, long n_t, long frame0,
                             float k_sigma, int cap);
lp_status trig_launch(const void *cand, int n_beams, int n_tec, long n_t,
                      long frame0, float k_sigma, lp_trig *out, int cap,
                      int *n_out, float *snr_out, int *best_tec,
                      float *sigma_out, void *work, hipStream_t st);

// Remap a linear block index so that consecutive logical blocks land on the
// same XCD (blocks are dealt round-robin over the 8 XCDs of the chip).
__device__ inline long xcd_remap(long bid, long nblocks) {
  const long nx = 8;
  if (nblocks < nx * 2) return bid;
  long per = nblocks / nx;           // full groups per XCD
  long full = per * nx;
  if (bid >= full) return bid;       // leftover tail keeps its index
  return (bid % nx) * per + bid / nx;
}

}  // namespace lp

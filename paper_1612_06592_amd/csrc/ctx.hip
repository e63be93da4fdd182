// Context, errors, sizing helpers and the cached chirp / synthesis tables.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "lp_internal.h"

namespace lp {

static thread_local std::string g_err;

lp_status set_error(lp_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

lp_status hip_fail(hipError_t e, const char *what) {
  return set_error(e == hipErrorOutOfMemory ? LP_ENOMEM : LP_EHIP,
                   "%s failed: %s", what, hipGetErrorString(e));
}

lp_status set_device(lp_ctx *ctx) {
  LP_HIP(hipSetDevice(ctx->device));
  return LP_OK;
}

lp_status check_band(const lp_band *band) {
  if (!band || band->n_sb <= 0 || !band->k)
    return set_error(LP_EINVAL, "band: n_sb must be > 0 and k non-NULL");
  if (band->n_sb > 511)
    return set_error(LP_EINVAL, "band: at most 511 subbands");
  if (band->M != kM || band->taps != kTaps)
    return set_error(LP_EINVAL, "band: M must be %d and taps %d", kM, kTaps);
  if (!(band->fs_hz > 0) || !(band->f0_hz >= 0))
    return set_error(LP_EINVAL, "band: bad f0/fs");
  for (int i = 0; i < band->n_sb; ++i) {
    int k = band->k[i];
    if (k < 1 || k > 511)
      return set_error(LP_EINVAL, "band: subband id %d outside 1..511", k);
    if (i > 0 && k <= band->k[i - 1])
      return set_error(LP_EINVAL, "band: subband ids must ascend strictly");
  }
  return LP_OK;
}

template <typename T>
static void put(std::vector<uint8_t> &v, const T &x) {
  const uint8_t *p = reinterpret_cast<const uint8_t *>(&x);
  v.insert(v.end(), p, p + sizeof(T));
}

static void put_band(std::vector<uint8_t> &v, const lp_band *b) {
  put(v, b->n_sb);
  for (int i = 0; i < b->n_sb; ++i) put(v, b->k[i]);
  put(v, b->f0_hz);
  put(v, b->fs_hz);
}

// ----------------------------------------------------------- plan cache

PlanBase *plan_find(lp_ctx *ctx, const std::vector<uint8_t> &key) {
  for (auto &p : ctx->plans)
    if (p->key == key) {
      p->tick = ++ctx->tick;
      ++p->refs;
      return p.get();
    }
  return nullptr;
}

// Frees the least recently used plan nobody holds; false if there is none.
// Its tables may still be read by queued kernels (or, in the bound buffer,
// be handed to a new plan at once), so the first eviction of a call waits
// for the device.
static bool evict_one(lp_ctx *ctx, bool *synced) {
  auto victim = ctx->plans.end();
  for (auto it = ctx->plans.begin(); it != ctx->plans.end(); ++it)
    if ((*it)->refs == 0 &&
        (victim == ctx->plans.end() || (*it)->tick < (*victim)->tick))
      victim = it;
  if (victim == ctx->plans.end()) return false;
  if (!*synced) {
    (void)hipDeviceSynchronize();
    *synced = true;
  }
  ctx->plans.erase(victim);
  return true;
}

lp_status plan_alloc(lp_ctx *ctx, PlanBase *p, DevBuf &b, size_t n) {
  n = std::max<size_t>(n, 1);
  if (!ctx->bound) {
    LP_HIP(hipMalloc(&b.p, n));
    b.n = n;
    p->bytes += n;
    return LP_OK;
  }
  size_t off = 0;
  bool synced = false;
  while (!ctx->const_arena.alloc(n, &off))
    if (!evict_one(ctx, &synced))
      return set_error(LP_ENOMEM,
                       "constant buffer: %zu bytes do not fit (%zu free, "
                       "the rest held by plans in use)",
                       n, ctx->const_arena.free_bytes());
  b.p = ctx->const_base + off;
  b.n = n;
  b.arena = &ctx->const_arena;
  b.off = off;
  p->bytes += Arena::round(n);
  return LP_OK;
}

lp_status plan_upload(PlanBase *p, DevBuf &b, const void *src, size_t n,
                      hipStream_t st) {
  const uint8_t *s8 = static_cast<const uint8_t *>(src);
  p->host.emplace_back(s8, s8 + n);
  LP_HIP(hipMemcpyAsync(b.p, p->host.back().data(), n, hipMemcpyHostToDevice,
                        st));
  return LP_OK;
}

lp_status plan_insert(lp_ctx *ctx, std::unique_ptr<PlanBase> p,
                      hipStream_t st) {
  LP_HIP(hipEventCreateWithFlags(&p->ready, hipEventDisableTiming));
  LP_HIP(hipEventRecord(p->ready, st));
  p->made_on = st;
  p->refs = 1;
  p->tick = ++ctx->tick;
  ctx->plans.push_back(std::move(p));
  bool synced = false;
  while (ctx->plans.size() > ctx->plan_max && evict_one(ctx, &synced)) {
  }
  return LP_OK;
}

lp_status plan_wait(PlanBase *p, hipStream_t st) {
  if (p->ready_seen.load(std::memory_order_acquire)) return LP_OK;
  hipError_t e = hipEventQuery(p->ready);
  if (e == hipSuccess) {
    p->ready_seen.store(true, std::memory_order_release);
    return LP_OK;
  }
  if (e != hipErrorNotReady) return hip_fail(e, "hipEventQuery(plan)");
  LP_HIP(hipStreamWaitEvent(st, p->ready, 0));
  return LP_OK;
}

void plan_release(lp_ctx *ctx, PlanBase *p) {
  std::lock_guard<std::mutex> g(ctx->mu);
  if (p->refs > 0) --p->refs;
}

// ---------------------------------------------------------------- chirp

// kappa = K_ion * 1e16 / c in s^-1 per TECU, K_ion = e^2/(8 pi^2 eps0 m_e)
// with CODATA 2018 constants.
static double kappa_per_tecu() {
  const double e = 1.602176634e-19, eps0 = 8.8541878128e-12,
               me = 9.1093837015e-31;
  const double kion = e * e / (8.0 * M_PI * M_PI * eps0 * me);
  return kion * 1e16 / kC;
}

// One thread per (trial, subband): the base phase kappa T / f_k is formed
// and range-reduced in FP64; only the reduced value and the (small)
// multiplier of the in-subband residual are rounded to FP32.
__global__ void dd_consts_kernel(const double *__restrict__ tec,
                                 const int *__restrict__ k, int n_tec,
                                 int n_sb, double f0, double df, double kap,
                                 float *__restrict__ base,
                                 float *__restrict__ afac,
                                 float *__restrict__ rfk) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_tec * n_sb) return;
  int j = i / n_sb, s = i % n_sb;
  double fk = f0 + (double)k[s] * df;
  double a = kap * tec[j] / fk;
  base[i] = (float)(a - rint(a));
  afac[i] = (float)a;
  if (j == 0) rfk[s] = (float)(df / (double)kNfft / fk);
}

// The trial-independent factor of the chirp phase, per subband and bin:
// g = x / (1 + x) with x = nu_q / f_k and nu_q = q_s (subband rate / N_fft).
__global__ void dd_ratio_kernel(const int *__restrict__ k, int n_sb, double f0,
                                double df, float *__restrict__ gq) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_sb * kNfft) return;
  const int s = (int)(i / kNfft), q = (int)(i % kNfft);
  const int qs = q < kNfft / 2 ? q : q - kNfft;
  const double fk = f0 + (double)k[s] * df;
  const double x = (double)qs * (df / (double)kNfft) / fk;
  gq[i] = (float)(x / (1.0 + x));
}

// Ratio of consecutive trials' chirps on a uniform grid of spacing dT, per
// subband and bin q (signed index q_s): exp(-2 pi i kappa dT / (f_k +
// nu_q)) (the delay term does not depend on the trial).  Formed in FP64,
// rounded once to FP32; one thread per entry.
__global__ void dd_rstep_kernel(double dT, const int *__restrict__ k,
                                int n_sb, double f0, double df, double kap,
                                float2 *__restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_sb * kNfft) return;
  const int s = (int)(i / kNfft), q = (int)(i % kNfft);
  const int qs = q < kNfft / 2 ? q : q - kNfft;
  const double f = f0 + (double)k[s] * df + (double)qs * (df / (double)kNfft);
  double ph = kap * dT / f;
  ph -= rint(ph);
  double sn, cs;
  sincospi(2.0 * ph, &sn, &cs);
  out[i] = make_float2((float)cs, (float)-sn);
}

lp_status get_dd_plan(lp_ctx *ctx, const lp_band *band, const double *tec,
                      int n_tec, hipStream_t st, PlanRef<DdPlan> &out) {
  std::vector<uint8_t> key(1, kPlanDd);
  put_band(key, band);
  put(key, n_tec);
  for (int j = 0; j < n_tec; ++j) put(key, tec[j]);
  std::lock_guard<std::mutex> g(ctx->mu);
  out.ctx = ctx;
  if (PlanBase *f = plan_find(ctx, key)) {
    out.p = static_cast<DdPlan *>(f);
    return LP_OK;
  }
  auto p = std::make_unique<DdPlan>();
  p->key = key;
  p->n_tec = n_tec;
  p->n_sb = band->n_sb;
  const int S = band->n_sb;
  const size_t js = (size_t)n_tec * S;
  std::vector<uint8_t> prm((size_t)n_tec * 8 + (size_t)S * 4);
  std::memcpy(prm.data(), tec, (size_t)n_tec * 8);
  std::memcpy(prm.data() + (size_t)n_tec * 8, band->k, (size_t)S * 4);
  lp_status rc;
  if ((rc = plan_alloc(ctx, p.get(), p->params, prm.size())) ||
      (rc = plan_upload(p.get(), p->params, prm.data(), prm.size(), st)) ||
      (rc = plan_alloc(ctx, p.get(), p->base, js * 4)) ||
      (rc = plan_alloc(ctx, p.get(), p->afac, js * 4)) ||
      (rc = plan_alloc(ctx, p.get(), p->rfk, (size_t)S * 4)) ||
      (rc = plan_alloc(ctx, p.get(), p->gq, (size_t)S * kNfft * 4)))
    return rc;
  // A uniform grid (at least two trials, T_t = T_0 + t dT) lets the kernel
  // step the chirp from trial to trial by a per-bin factor.
  double dT = 0.0;
  if (n_tec >= 2) {
    dT = (tec[n_tec - 1] - tec[0]) / (n_tec - 1);
    bool uni = true;
    for (int j = 0; j < n_tec; ++j)
      if (std::fabs(tec[j] - (tec[0] + j * dT)) >
          1e-9 * std::max(1.0, std::fabs(tec[n_tec - 1])))
        uni = false;
    p->uniform = uni;
  }
  if (p->uniform && (rc = plan_alloc(ctx, p.get(), p->rstep,
                                    (size_t)S * kNfft * sizeof(float2))))
    return rc;
  const double *dtec = p->params.as<const double>();
  const int *dk = reinterpret_cast<const int *>(p->params.as<const char>() +
                                                (size_t)n_tec * 8);
  int n = (int)js;
  hipLaunchKernelGGL(dd_consts_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     st, dtec, dk, n_tec, S, band->f0_hz, band->fs_hz / kM,
                     kappa_per_tecu(), p->base.as<float>(),
                     p->afac.as<float>(), p->rfk.as<float>());
  LP_HIP(hipGetLastError());
  const long ng = (long)S * kNfft;
  hipLaunchKernelGGL(dd_ratio_kernel, dim3((unsigned)((ng + 255) / 256)),
                     dim3(256), 0, st, dk, S, band->f0_hz, band->fs_hz / kM,
                     p->gq.as<float>());
  LP_HIP(hipGetLastError());
  if (p->uniform) {
    hipLaunchKernelGGL(dd_rstep_kernel, dim3((unsigned)((ng + 255) / 256)),
                       dim3(256), 0, st, dT, dk, S, band->f0_hz,
                       band->fs_hz / kM, kappa_per_tecu(),
                       p->rstep.as<float2>());
    LP_HIP(hipGetLastError());
  }
  DdPlan *raw = p.get();
  if ((rc = plan_insert(ctx, std::move(p), st))) return rc;
  out.p = raw;
  return LP_OK;
}

// ------------------------------------------------------------ synthesis

static double bessel_i0(double x) {
  // Power series sum_m ((x/2)^m / m!)^2, summed until the terms vanish.
  double term = 1.0, sum = 1.0, h = 0.5 * x;
  for (int m = 1; m < 400 && term > sum * 1e-18; ++m) {
    term *= (h / m) * (h / m);
    sum += term;
  }
  return sum;
}

lp_status get_syn_plan(lp_ctx *ctx, const lp_band *band, hipStream_t st,
                       PlanRef<SynPlan> &out) {
  std::vector<uint8_t> key(1, kPlanSyn);
  put(key, band->kaiser_beta);
  put(key, band->n_sb);
  for (int i = 0; i < band->n_sb; ++i) put(key, band->k[i]);
  std::lock_guard<std::mutex> g(ctx->mu);
  out.ctx = ctx;
  if (PlanBase *f = plan_find(ctx, key)) {
    out.p = static_cast<SynPlan *>(f);
    return LP_OK;
  }
  auto p = std::make_unique<SynPlan>();
  p->key = key;
  // Prototype h (Kaiser-windowed sinc, unit sum) in FP64; taps g = M h.
  const int L = kM * kTaps;
  std::vector<double> h(L);
  double i0b = bessel_i0(band->kaiser_beta), sum = 0.0;
  for (int l = 0; l < L; ++l) {
    double u = 2.0 * l / (L - 1) - 1.0;
    double w = bessel_i0(band->kaiser_beta * std::sqrt(std::max(0.0, 1.0 - u * u))) / i0b;
    double xs = (l - 0.5 * (L - 1)) / kM;
    double sc = std::sin(M_PI * xs) / (M_PI * xs);
    h[l] = w * sc;
    sum += h[l];
  }
  std::vector<float> g32(L), g2(L);
  for (int l = 0; l < L; ++l) {
    g32[l] = (float)(kM * h[l] / sum);
    g2[l] = 2.f * g32[l];
  }
  std::vector<int16_t> bm(512, -1);
  for (int i = 0; i < band->n_sb; ++i) bm[band->k[i]] = (int16_t)i;
  p->kmax = 0;
  for (int i = 0; i < band->n_sb; ++i) p->kmax = std::max(p->kmax, (int)band->k[i]);
  std::vector<int16_t> kb(band->n_sb);
  for (int i = 0; i < band->n_sb; ++i) kb[i] = (int16_t)band->k[i];
  lp_status rc;
  if ((rc = plan_alloc(ctx, p.get(), p->taps, L * 4)) ||
      (rc = plan_upload(p.get(), p->taps, g32.data(), L * 4, st)) ||
      (rc = plan_alloc(ctx, p.get(), p->taps2, L * 4)) ||
      (rc = plan_upload(p.get(), p->taps2, g2.data(), L * 4, st)) ||
      (rc = plan_alloc(ctx, p.get(), p->binmap, 512 * 2)) ||
      (rc = plan_upload(p.get(), p->binmap, bm.data(), 512 * 2, st)) ||
      (rc = plan_alloc(ctx, p.get(), p->kbin, band->n_sb * 2)) ||
      (rc = plan_upload(p.get(), p->kbin, kb.data(), band->n_sb * 2, st)))
    return rc;
  SynPlan *raw = p.get();
  if ((rc = plan_insert(ctx, std::move(p), st))) return rc;
  out.p = raw;
  return LP_OK;
}

}  // namespace lp

using namespace lp;

extern "C" {

const char *lp_last_error(void) { return g_err.c_str(); }

const char *lp_version(void) { return "liblp 0.1 gfx950"; }

lp_status lp_ctx_create(int32_t hip_device, lp_ctx **out) {
  if (!out) return set_error(LP_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || hip_device < 0 || hip_device >= n)
    return set_error(LP_EHIP, "no HIP device %d (count %d)", hip_device, n);
  auto ctx = std::make_unique<lp_ctx>();
  ctx->device = hip_device;
  LP_HIP(hipSetDevice(hip_device));
  LP_HIP(hipDeviceGetAttribute(&ctx->n_cu,
                               hipDeviceAttributeMultiprocessorCount,
                               hip_device));
  if (ctx->n_cu <= 0) ctx->n_cu = 1;
  std::vector<float2> tw(4096);
  for (int i = 0; i < 4096; ++i) {
    double a = -2.0 * M_PI * i / 4096.0;
    tw[i] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  LP_HIP(hipMalloc(&ctx->tw4096.p, 4096 * sizeof(float2)));
  LP_HIP(hipMemcpy(ctx->tw4096.p, tw.data(), 4096 * sizeof(float2),
                   hipMemcpyHostToDevice));
  lp_status rc = trig_scratch_attach(hip_device);
  if (rc) return rc;
  *out = ctx.release();
  return LP_OK;
}

lp_status lp_ctx_bind_const(lp_ctx *ctx, void *dev, size_t bytes) {
  if (!ctx) return set_error(LP_EINVAL, "lp_ctx_bind_const: NULL ctx");
  if (dev && (bytes < 256 || reinterpret_cast<uintptr_t>(dev) % 256))
    return set_error(LP_EINVAL, "lp_ctx_bind_const: the buffer must be "
                                "256-byte aligned and at least 256 bytes");
  lp_status rc;
  if ((rc = set_device(ctx))) return rc;
  std::lock_guard<std::mutex> g(ctx->mu);
  for (auto &p : ctx->plans)
    if (p->refs > 0)
      return set_error(LP_EINVAL, "lp_ctx_bind_const: plans are in use "
                                  "(open serving streams or calls)");
  if (!ctx->plans.empty()) {
    LP_HIP(hipDeviceSynchronize());
    ctx->plans.clear();
  }
  ctx->bound = dev != nullptr;
  ctx->const_base = static_cast<char *>(dev);
  ctx->const_arena.init(dev ? bytes : 0);
  return LP_OK;
}

lp_status lp_ctx_plan_cache(lp_ctx *ctx, int32_t max_plans) {
  if (!ctx || max_plans < 0)
    return set_error(LP_EINVAL, "lp_ctx_plan_cache: bad arguments");
  lp_status rc;
  if ((rc = set_device(ctx))) return rc;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->plan_max = (size_t)max_plans;
  bool synced = false;
  while (ctx->plans.size() > ctx->plan_max && evict_one(ctx, &synced)) {
  }
  return LP_OK;
}

lp_status lp_ctx_plan_stats(lp_ctx *ctx, int32_t *n_plans, int32_t *n_held,
                            size_t *device_bytes) {
  if (!ctx) return set_error(LP_EINVAL, "lp_ctx_plan_stats: NULL ctx");
  std::lock_guard<std::mutex> g(ctx->mu);
  int held = 0;
  size_t bytes = 0;
  for (auto &p : ctx->plans) {
    held += p->refs > 0;
    bytes += p->bytes;
  }
  if (n_plans) *n_plans = (int32_t)ctx->plans.size();
  if (n_held) *n_held = held;
  if (device_bytes) *device_bytes = bytes;
  return LP_OK;
}

void lp_ctx_destroy(lp_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  delete ctx;
}

size_t lp_beam_bytes(int32_t n_beams, int32_t n_sb, int64_t n_t) {
  return (size_t)n_beams * n_sb * n_t * 8;
}
size_t lp_dd_state_bytes(int32_t n_beams, int32_t n_sb) {
  return (size_t)n_beams * n_sb * kHist * 8;
}
size_t lp_dd_bytes(int32_t n_beams, int32_t n_tec, int32_t n_sb,
                   int64_t n_t) {
  return (size_t)n_beams * n_tec * n_sb * n_t * 8;
}
size_t lp_syn_state_bytes(int32_t n_series, int32_t n_sb) {
  return (size_t)n_series * n_sb * kSynHist * 8;
}
size_t lp_cand_bytes(int32_t n_series, int64_t n_t) {
  return (size_t)n_series * n_t * 8 + (size_t)n_series * (n_t / 16) * 4;
}

}  // extern "C"

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

lp_status get_dd_plan(lp_ctx *ctx, const lp_band *band, const double *tec,
                      int n_tec, DdPlan **out) {
  std::vector<uint8_t> key;
  put_band(key, band);
  put(key, n_tec);
  for (int j = 0; j < n_tec; ++j) put(key, tec[j]);
  std::lock_guard<std::mutex> g(ctx->mu);
  for (auto &p : ctx->dd)
    if (p->key == key) {
      *out = p.get();
      return LP_OK;
    }
  auto p = std::make_unique<DdPlan>();
  p->key = key;
  p->n_tec = n_tec;
  p->n_sb = band->n_sb;
  size_t js = (size_t)n_tec * band->n_sb;
  LP_HIP(hipMalloc(&p->base.p, js * 4));
  LP_HIP(hipMalloc(&p->afac.p, js * 4));
  LP_HIP(hipMalloc(&p->rfk.p, band->n_sb * 4));
  LP_HIP(hipMalloc(&p->gq.p, (size_t)band->n_sb * kNfft * 4));
  DevBuf dtec, dk;
  LP_HIP(hipMalloc(&dtec.p, n_tec * 8));
  LP_HIP(hipMalloc(&dk.p, band->n_sb * 4));
  LP_HIP(hipMemcpy(dtec.p, tec, n_tec * 8, hipMemcpyHostToDevice));
  LP_HIP(hipMemcpy(dk.p, band->k, band->n_sb * 4, hipMemcpyHostToDevice));
  int n = (int)js;
  hipLaunchKernelGGL(dd_consts_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     0, dtec.as<double>(), dk.as<int>(), n_tec, band->n_sb,
                     band->f0_hz, band->fs_hz / kM, kappa_per_tecu(),
                     p->base.as<float>(), p->afac.as<float>(),
                     p->rfk.as<float>());
  LP_HIP(hipGetLastError());
  const long ng = (long)band->n_sb * kNfft;
  hipLaunchKernelGGL(dd_ratio_kernel, dim3((unsigned)((ng + 255) / 256)),
                     dim3(256), 0, 0, dk.as<int>(), band->n_sb, band->f0_hz,
                     band->fs_hz / kM, p->gq.as<float>());
  LP_HIP(hipGetLastError());
  LP_HIP(hipDeviceSynchronize());
  *out = p.get();
  ctx->dd.push_back(std::move(p));
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

lp_status get_syn_plan(lp_ctx *ctx, const lp_band *band, SynPlan **out) {
  std::vector<uint8_t> key;
  put(key, band->kaiser_beta);
  put(key, band->n_sb);
  for (int i = 0; i < band->n_sb; ++i) put(key, band->k[i]);
  std::lock_guard<std::mutex> g(ctx->mu);
  for (auto &p : ctx->syn)
    if (p->key == key) {
      *out = p.get();
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
  std::vector<float> g32(L);
  for (int l = 0; l < L; ++l) g32[l] = (float)(kM * h[l] / sum);
  std::vector<int16_t> bm(512, -1);
  for (int i = 0; i < band->n_sb; ++i) bm[band->k[i]] = (int16_t)i;
  p->kmax = 0;
  for (int i = 0; i < band->n_sb; ++i) p->kmax = std::max(p->kmax, (int)band->k[i]);
  LP_HIP(hipMalloc(&p->taps.p, L * 4));
  LP_HIP(hipMalloc(&p->binmap.p, 512 * 2));
  LP_HIP(hipMemcpy(p->taps.p, g32.data(), L * 4, hipMemcpyHostToDevice));
  for (int l = 0; l < L; ++l) g32[l] *= 2.f;
  LP_HIP(hipMalloc(&p->taps2.p, L * 4));
  LP_HIP(hipMemcpy(p->taps2.p, g32.data(), L * 4, hipMemcpyHostToDevice));
  LP_HIP(hipMemcpy(p->binmap.p, bm.data(), 512 * 2, hipMemcpyHostToDevice));
  std::vector<int16_t> kb(band->n_sb);
  for (int i = 0; i < band->n_sb; ++i) kb[i] = (int16_t)band->k[i];
  LP_HIP(hipMalloc(&p->kbin.p, band->n_sb * 2));
  LP_HIP(hipMemcpy(p->kbin.p, kb.data(), band->n_sb * 2, hipMemcpyHostToDevice));
  *out = p.get();
  ctx->syn.push_back(std::move(p));
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
  *out = ctx.release();
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
size_t lp_trigger_work_bytes(int32_t n_beams, int32_t n_tec) {
  size_t ns = (size_t)n_beams * n_tec;
  return ns * 16                                   // count, sigma, peak, pad
         + ns * kTrigPerSeries * 16                // per-series lists
         + (size_t)n_beams * 16                    // per-beam counts
         + (size_t)n_beams * n_tec * kTrigPerSeries * sizeof(lp_trig);
}

}  // extern "C"

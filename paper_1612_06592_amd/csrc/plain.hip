// Plain FP32 comparator of the de-dispersion and synthesis stages: the same
// arithmetic as dd_kernel / syn_kernel, organised the straightforward way.
// Every intermediate (overlap-save buffers, spectra, each radix-2 FFT pass,
// the filtered series, the envelope, the real series) is a full array in
// HBM, and each step is its own kernel.  It is the baseline the fused path
// is measured against, and its results equal the fused path's to FP32
// rounding.  Work is processed in groups of beams / series that fit the
// caller's workspace.
#include <algorithm>
#include <cmath>

#include "fft_dev.h"
#include "lp_internal.h"

namespace lp {

struct PlainCand {
  float emax;
  int arg;
};

// One radix-2 Stockham pass over `batch` transforms of length N (a power of
// two): butterfly j reads src[j], src[j + N/2], twiddles the second by
// exp(s 2 pi i (j mod Ns) / (2 Ns)) and writes (j / Ns) 2 Ns + j mod Ns
// and + Ns.
__global__ void pl_fft_pass(const float2 *__restrict__ src,
                            float2 *__restrict__ dst, int N, int Ns, int inv,
                            long batch, const float2 *__restrict__ tw) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long half = N / 2;
  if (i >= batch * half) return;
  long b = i / half;
  int j = (int)(i % half);
  const float2 *s = src + b * N;
  float2 *d = dst + b * N;
  float2 v0 = s[j], v1 = s[j + half];
  int k = (j % Ns) * (4096 / (2 * Ns));   // table index of the angle
  float2 w = tw[k];
  if (inv) w.y = -w.y;
  v1 = cmul(v1, w);
  int o = (j / Ns) * 2 * Ns + (j % Ns);
  d[o] = cadd(v0, v1);
  d[o + Ns] = csub(v0, v1);
}

// Transform `batch` arrays of length N in place (via `tmp`): log2 N passes.
static lp_status fft_global(float2 *buf, float2 *tmp, int N, bool inv,
                            long batch, const float2 *tw, hipStream_t st) {
  float2 *a = buf, *b = tmp;
  for (int Ns = 1; Ns < N; Ns *= 2) {
    long n = batch * (N / 2);
    hipLaunchKernelGGL(pl_fft_pass, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, st, a, b, N, Ns, inv ? 1 : 0, batch, tw);
    float2 *t = a;
    a = b;
    b = t;
  }
  LP_HIP(hipGetLastError());
  if (a != buf)
    LP_HIP(hipMemcpyAsync(buf, a, (size_t)batch * N * sizeof(float2),
                          hipMemcpyDeviceToDevice, st));
  return LP_OK;
}

// ------------------------------------------------------- de-dispersion

// U[b][s][h][0..4096) = [2048 previous samples | 2048 new samples].
__global__ void pl_dd_gather(const float2 *__restrict__ y,
                             const float2 *__restrict__ tail,
                             float2 *__restrict__ U, int n_sb, long n_t,
                             int n_hop, long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int q = (int)(i % 4096);
  long bsh = i / 4096;
  int h = (int)(bsh % n_hop);
  long bs = bsh / n_hop;
  long t = (long)h * kHop - kHist + q;
  U[i] = (t < 0) ? tail[bs * kHist + (kHist + t)] : y[bs * n_t + t];
}

// V = U * chirp_j (the same phase formula as the fused kernel).
__global__ void pl_dd_chirp(const float2 *__restrict__ U,
                            float2 *__restrict__ V,
                            const float *__restrict__ base,
                            const float *__restrict__ afac,
                            const float *__restrict__ rfk, int jt, int n_sb,
                            int n_hop, long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int q = (int)(i % 4096);
  int s = (int)((i / 4096 / n_hop) % n_sb);
  int qs = q < 2048 ? q : q - 4096;
  float x = (float)qs * rfk[s];
  float A = afac[jt * n_sb + s];
  float c = base[jt * n_sb + s] - A * x / (1.0f + x) + 0.25f * (float)(qs & 3);
  c -= rintf(c);
  float sn, cs;
  sincospif(2.0f * c, &sn, &cs);
  V[i] = cmul(U[i], make_float2(cs, -sn));
}

// d[b][j][s][h*2048 + i] = V[b][s][h][2048 + i] / 4096.
__global__ void pl_dd_extract(const float2 *__restrict__ V,
                              float2 *__restrict__ d, int jt, int n_tec,
                              int n_sb, long n_t, int n_hop, int b0,
                              long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int k = (int)(i % kHop);
  long bsh = i / kHop;
  int h = (int)(bsh % n_hop);
  long bs = bsh / n_hop;
  int s = (int)(bs % n_sb);
  int b = b0 + (int)(bs / n_sb);
  float2 v = V[bsh * 4096 + kHist + k];
  d[(((long)b * n_tec + jt) * n_sb + s) * n_t + (long)h * kHop + k] =
      make_float2(v.x * (1.0f / 4096.0f), v.y * (1.0f / 4096.0f));
}

__global__ void pl_dd_tail(const float2 *__restrict__ y,
                           float2 *__restrict__ tail, long n_t, long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  long bs = i / kHist;
  int k = (int)(i % kHist);
  tail[i] = y[bs * n_t + (n_t - kHist) + k];
}

// --------------------------------------------------------------- synthesis

// X[q][f][0..1024): spectrum of frame f - 15 (f < 15: history), d at bin k.
__global__ void pl_syn_spectrum(const float2 *__restrict__ d,
                                const float2 *__restrict__ hist,
                                const short *__restrict__ binmap,
                                float2 *__restrict__ X, int n_sb, long n_t,
                                int q0, long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int k = (int)(i % 1024);
  long qf = i / 1024;
  long nf = n_t + 15;
  long f = qf % nf;
  int q = q0 + (int)(qf / nf);
  long m = f - 15;
  float2 v = make_float2(0.f, 0.f);
  int si = k < 512 ? binmap[k] : -1;
  if (si >= 0)
    v = (m >= 0) ? d[((long)q * n_sb + si) * n_t + m]
                 : hist[((long)q * n_sb + si) * kSynHist + (kSynHist + m)];
  X[i] = v;
}

// z[q][m][n] = sum_t g[t][n] Z[q][m + 15 - t][n].
__global__ void pl_syn_fir(const float2 *__restrict__ Z,
                           const float *__restrict__ taps,
                           float2 *__restrict__ z, long n_t, long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int n = (int)(i % 1024);
  long qm = i / 1024;
  long m = qm % n_t;
  long q = qm / n_t;
  const float2 *Zq = Z + q * (n_t + 15) * 1024;
  float zr = 0.f, zi = 0.f;
  for (int t = 0; t < 16; ++t) {
    float2 w = Zq[(m + 15 - t) * 1024 + n];
    float g = taps[t * 1024 + n];
    zr = fmaf(g, w.x, zr);
    zi = fmaf(g, w.y, zi);
  }
  z[i] = make_float2(zr, zi);
}

// e = |2 z|, xr = 2 Re z.
__global__ void pl_envelope(const float2 *__restrict__ z,
                            float *__restrict__ e, float *__restrict__ xr,
                            long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  float2 v = z[i];
  e[i] = sqrtf(4.f * (v.x * v.x + v.y * v.y));
  xr[i] = 2.f * v.x;
}

// One wave per frame: envelope maximum (lowest n on ties); one wave per
// 16 frames: sum of xr^2 over valid frames.
__global__ void pl_windows(const float *__restrict__ e,
                           PlainCand *__restrict__ cand, long n_t, int q0,
                           long n_frames) {
  long f = (long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  int lane = threadIdx.x & 63;
  if (f >= n_frames) return;
  const float *ef = e + f * 1024;
  float bv = -1.f;
  int bi = 0;
  for (int i = 0; i < 16; ++i) {
    float v = ef[lane + 64 * i];
    if (v > bv) {
      bv = v;
      bi = lane + 64 * i;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    float ov = __shfl_xor(bv, off);
    int oi = __shfl_xor(bi, off);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    long q = q0 + f / n_t, m = f % n_t;
    PlainCand c;
    c.emax = bv;
    c.arg = bi;
    cand[q * n_t + m] = c;
  }
}

__global__ void pl_sigma_partials(const float *__restrict__ xr,
                                  float *__restrict__ psum, long n_t, int q0,
                                  long frame0, long warm, long n_chunks) {
  long c = (long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  int lane = threadIdx.x & 63;
  if (c >= n_chunks) return;
  long per_q = n_t / 16;
  long q = c / per_q, m0 = (c % per_q) * 16;
  float acc = 0.f;
  for (int f = 0; f < 16; ++f) {
    if (frame0 + m0 + f < warm) continue;
    const float *x = xr + (q * n_t + m0 + f) * 1024;
    for (int i = 0; i < 16; ++i) {
      float v = x[lane + 64 * i];
      acc = fmaf(v, v, acc);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) psum[(q0 + q) * per_q + m0 / 16] = acc;
}

__global__ void pl_syn_hist(const float2 *__restrict__ d,
                            float2 *__restrict__ hist, long n_t,
                            long total) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  long qs = i / kSynHist;
  int f = (int)(i % kSynHist);
  hist[i] = d[qs * n_t + (n_t - kSynHist) + f];
}

static dim3 grid_of(long n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace lp

using namespace lp;

extern "C" {

size_t lp_plain_work_bytes(int32_t n_beams, int32_t n_tec, int32_t n_sb,
                           int64_t n_t) {
  // De-dispersion of one beam: U, V, scratch (4096 per hop each).
  size_t dd = (size_t)n_sb * (n_t / kHop) * 4096 * 8 * 3;
  // Synthesis of one series: X, scratch ((n_t + 15) frames), z, e, xr.
  size_t syn = (size_t)(n_t + 15) * 1024 * 8 * 2 + (size_t)n_t * 1024 * 16;
  (void)n_beams;
  (void)n_tec;
  return dd > syn ? dd : syn;
}

lp_status lp_dedisperse_plain(lp_ctx *ctx, const lp_band *band,
                              const double *tec_tecu, int32_t n_tec,
                              const void *y, int32_t n_beams, int64_t n_t,
                              void *tail, int32_t flags, void *d, void *work,
                              size_t work_bytes, void *hip_stream) {
  if (!ctx || !tec_tecu || !y || !tail || !d || !work)
    return set_error(LP_EINVAL, "lp_dedisperse_plain: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (n_tec <= 0 || n_beams <= 0 || n_t <= 0 || n_t % kHop)
    return set_error(LP_EINVAL, "lp_dedisperse_plain: bad sizes");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<DdPlan> p;
  if ((rc = get_dd_plan(ctx, band, tec_tecu, n_tec, st, p)) ||
      (rc = plan_wait(p.get(), st)))
    return rc;
  const int S = band->n_sb, n_hop = (int)(n_t / kHop);
  const size_t per_beam = (size_t)S * n_hop * 4096 * 8;
  const int grp = (int)std::min<size_t>(n_beams, work_bytes / (3 * per_beam));
  if (grp < 1)
    return set_error(LP_EINVAL, "lp_dedisperse_plain: workspace too small");
  float2 *U = static_cast<float2 *>(work);
  float2 *V = U + (size_t)grp * S * n_hop * 4096;
  float2 *T = V + (size_t)grp * S * n_hop * 4096;
  const float2 *yy = static_cast<const float2 *>(y);
  float2 *tl = static_cast<float2 *>(tail);
  for (int b0 = 0; b0 < n_beams; b0 += grp) {
    int nb = std::min(grp, n_beams - b0);
    long nU = (long)nb * S * n_hop * 4096;
    hipLaunchKernelGGL(pl_dd_gather, grid_of(nU), dim3(256), 0, st,
                       yy + (long)b0 * S * n_t, tl + (long)b0 * S * kHist, U,
                       S, (long)n_t, n_hop, nU);
    if ((rc = fft_global(U, T, 4096, false, (long)nb * S * n_hop,
                         ctx->tw4096.as<const float2>(), st)))
      return rc;
    for (int jt = 0; jt < n_tec; ++jt) {
      hipLaunchKernelGGL(pl_dd_chirp, grid_of(nU), dim3(256), 0, st, U, V,
                         p->base.as<const float>(), p->afac.as<const float>(),
                         p->rfk.as<const float>(), jt, S, n_hop, nU);
      if ((rc = fft_global(V, T, 4096, true, (long)nb * S * n_hop,
                           ctx->tw4096.as<const float2>(), st)))
        return rc;
      long nd = (long)nb * S * n_hop * kHop;
      hipLaunchKernelGGL(pl_dd_extract, grid_of(nd), dim3(256), 0, st, V,
                         static_cast<float2 *>(d), jt, n_tec, S, (long)n_t,
                         n_hop, b0, nd);
    }
  }
  if (!(flags & LP_DD_KEEP_TAIL)) {
    long nt = (long)n_beams * S * kHist;
    hipLaunchKernelGGL(pl_dd_tail, grid_of(nt), dim3(256), 0, st, yy, tl,
                       (long)n_t, nt);
  }
  LP_HIP(hipGetLastError());
  return LP_OK;
}

lp_status lp_synthesize_plain(lp_ctx *ctx, const lp_band *band, const void *d,
                              int32_t n_series, int64_t n_t, int64_t frame0,
                              void *hist, float *x_out, void *cand, void *work,
                              size_t work_bytes, void *hip_stream) {
  if (!ctx || !d || !hist || !cand || !work)
    return set_error(LP_EINVAL, "lp_synthesize_plain: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (n_series <= 0 || n_t <= 0 || n_t % kHop || frame0 < 0)
    return set_error(LP_EINVAL, "lp_synthesize_plain: bad sizes");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<SynPlan> p;
  if ((rc = get_syn_plan(ctx, band, st, p)) || (rc = plan_wait(p.get(), st)))
    return rc;
  const int S = band->n_sb;
  const size_t nX = (size_t)(n_t + 15) * 1024, nz = (size_t)n_t * 1024;
  const size_t per = nX * 8 * 2 + nz * 16;
  const int grp = (int)std::min<size_t>(n_series, work_bytes / per);
  if (grp < 1)
    return set_error(LP_EINVAL, "lp_synthesize_plain: workspace too small");
  char *w = static_cast<char *>(work);
  float2 *X = reinterpret_cast<float2 *>(w);
  float2 *T = X + (size_t)grp * nX;
  float2 *z = T + (size_t)grp * nX;
  float *e = reinterpret_cast<float *>(z + (size_t)grp * nz);
  float *xr = e + (size_t)grp * nz;
  char *cb = static_cast<char *>(cand);
  PlainCand *cd = reinterpret_cast<PlainCand *>(cb);
  float *ps = reinterpret_cast<float *>(cb + (size_t)n_series * n_t * 8);
  for (int q0 = 0; q0 < n_series; q0 += grp) {
    int nq = std::min(grp, n_series - q0);
    long n1 = (long)nq * nX;
    hipLaunchKernelGGL(pl_syn_spectrum, grid_of(n1), dim3(256), 0, st,
                       static_cast<const float2 *>(d),
                       static_cast<const float2 *>(hist),
                       p->binmap.as<const short>(), X, S, (long)n_t, q0, n1);
    if ((rc = fft_global(X, T, 1024, true, (long)nq * (n_t + 15),
                         ctx->tw4096.as<const float2>(), st)))
      return rc;
    long n2 = (long)nq * nz;
    hipLaunchKernelGGL(pl_syn_fir, grid_of(n2), dim3(256), 0, st, X,
                       p->taps.as<const float>(), z, (long)n_t, n2);
    float *xdst = x_out ? x_out + (size_t)q0 * nz : xr;
    hipLaunchKernelGGL(pl_envelope, grid_of(n2), dim3(256), 0, st, z, e,
                       xdst, n2);
    long nfr = (long)nq * n_t;
    hipLaunchKernelGGL(pl_windows, dim3((unsigned)((nfr + 3) / 4)), dim3(256),
                       0, st, e, cd, (long)n_t, q0, nfr);
    long nch = (long)nq * (n_t / 16);
    hipLaunchKernelGGL(pl_sigma_partials, dim3((unsigned)((nch + 3) / 4)),
                       dim3(256), 0, st, xdst, ps, (long)n_t, q0,
                       (long)frame0, (long)(kDelay + kTaps), nch);
  }
  long nh = (long)n_series * S * kSynHist;
  hipLaunchKernelGGL(pl_syn_hist, grid_of(nh), dim3(256), 0, st,
                     static_cast<const float2 *>(d), static_cast<float2 *>(hist),
                     (long)n_t, nh);
  LP_HIP(hipGetLastError());
  return LP_OK;
}

}  // extern "C"

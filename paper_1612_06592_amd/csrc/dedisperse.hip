// Ionospheric de-dispersion (Winchen et al. 2016, Sec. 3, dispersion
// paragraph): per beam and subband the series is multiplied in the
// frequency domain by the complex weight of the trial STEC.  Overlap-save:
// each hop of 2048 new samples forms a 4096-point buffer with the previous
// 2048 samples, is transformed once, and for every trial is multiplied by
//   exp(-2 pi i [kappa T / (f_k + nu_q) + q_s D / 4096])
// and transformed back; the last 2048 outputs are kept.
//
// One 256-thread workgroup per (beam, subband, hop).  Each thread owns 16
// points; the 4096-point transform is three radix-16 Stockham passes with
// two exchanges through a padded 34 KB LDS tile.  The forward spectrum
// stays in registers across all trials.
#include <cmath>

#include "fft_dev.h"
#include "lp_internal.h"

namespace lp {

constexpr int kDdThreads = 256;
constexpr int kDdLds = 4096 + 128;  // slot of element 4095 is 4222

// 4096-point transform of v[r] = in[j + 256 r] (j = thread); on return
// v[r] = out[j + 256 r].  Unnormalised; INV selects exp(+2 pi i ...).
// Twiddles exp(-2 pi i n / 4096) from two small LDS tables:
// coarse[c] = w^(16 c) (c < 256), fine[f] = w^f (f < 16).
template <bool INV>
__device__ __forceinline__ float2 tw4096_lds(const float2 *coarse,
                                             const float2 *fine, int n) {
  float2 w = cmul(coarse[(n >> 4) & 255], fine[n & 15]);
  return INV ? make_float2(w.x, -w.y) : w;
}

// v[r] *= w^r (r = 1..15), the powers formed by a product tree of depth 4
// and each used as soon as it exists (few live registers, short chains).
__device__ __forceinline__ void pow16_twiddle(float2 *v, const float2 w1) {
  const float2 w2 = cmul(w1, w1), w4 = cmul(w2, w2), w8 = cmul(w4, w4);
  const float2 w3 = cmul(w2, w1);
  v[1] = cmul(v[1], w1);
  v[2] = cmul(v[2], w2);
  v[3] = cmul(v[3], w3);
  v[4] = cmul(v[4], w4);
  v[5] = cmul(v[5], cmul(w4, w1));
  v[6] = cmul(v[6], cmul(w4, w2));
  const float2 w7 = cmul(w4, w3);
  v[7] = cmul(v[7], w7);
  v[8] = cmul(v[8], w8);
  v[9] = cmul(v[9], cmul(w8, w1));
  v[10] = cmul(v[10], cmul(w8, w2));
  v[11] = cmul(v[11], cmul(w8, w3));
  v[12] = cmul(v[12], cmul(w8, w4));
  v[13] = cmul(v[13], cmul(w8, cmul(w4, w1)));
  v[14] = cmul(v[14], cmul(w8, cmul(w4, w2)));
  v[15] = cmul(v[15], cmul(w8, w7));
}

template <bool INV>
__device__ __forceinline__ void fft4096(float2 *v, float2 *lds,
                                        const float2 *coarse,
                                        const float2 *fine, int j) {
  // Element e sits at slot e + e / 32 (one pad slot per 32: every access
  // pattern below puts the 64 lanes' 8-byte words evenly on the banks, for
  // 32 or 64 banks).  In closed form (j < 256, r < 16):
  //   16 j + r -> 16 j + j / 2 + r,  j + 256 r -> j + j / 32 + 264 r,
  //   (j / 16) 256 + j mod 16 + 16 r -> (j / 16) 264 + j mod 16 + 16 r + r / 2.
  const int sj = j + (j >> 5);
  // Pass 0 (Ns = 1): no twiddle; write to (16 j + r).
  dft16<INV>(v);
  __syncthreads();
  {
    const int b0 = 16 * j + (j >> 1);
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[b0 + r] = v[r];
  }
  __syncthreads();
  // Pass 1 (Ns = 16).
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[sj + 264 * r];
  {
    const float2 w = coarse[j & 15];  // angle 2 pi (j mod 16) / 256
    pow16_twiddle(v, INV ? make_float2(w.x, -w.y) : w);
  }
  dft16<INV>(v);
  __syncthreads();
  {
    const int b2 = (j >> 4) * 264 + (j & 15);
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[b2 + 16 * r + (r >> 1)] = v[r];
  }
  __syncthreads();
  // Pass 2 (Ns = 256): output index j + 256 r stays in registers.
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[sj + 264 * r];
  pow16_twiddle(v, tw4096_lds<INV>(coarse, fine, j));
  dft16<INV>(v);
}

__global__ __launch_bounds__(kDdThreads)
__attribute__((amdgpu_waves_per_eu(4, 8))) void dd_kernel(
    const float2 *__restrict__ y, float2 *__restrict__ tail, int update_tail,
    float2 *__restrict__ d, const float2 *__restrict__ tw,
    const float *__restrict__ base, const float *__restrict__ afac,
    const float *__restrict__ gq, int n_sb, int n_tec, long n_t, int n_hop,
    long n_blocks) {
  __shared__ float2 lds[kDdLds];
  __shared__ float2 coarse[256], fine[16];
  coarse[threadIdx.x] = tw[16 * threadIdx.x];
  if (threadIdx.x < 16) fine[threadIdx.x] = tw[threadIdx.x];
  // (the barrier inside the first transform orders these before use)
  const long bid = xcd_remap(blockIdx.x, n_blocks);
  const int h = (int)(bid % n_hop);
  const long bs = bid / n_hop;          // beam * n_sb + subband
  const int s = (int)(bs % n_sb);
  const int b = (int)(bs / n_sb);
  const int j = threadIdx.x;
  const float2 *ys = y + bs * n_t;
  float2 *tl = tail + bs * kHist;
  const long hs = (long)h * kHop;

  float2 v[16];
#pragma unroll
  for (int r = 0; r < 8; ++r)
    v[r] = (h == 0) ? tl[j + 256 * r] : ys[hs - kHist + j + 256 * r];
#pragma unroll
  for (int r = 8; r < 16; ++r) v[r] = ys[hs + j + 256 * (r - 8)];

  fft4096<false>(v, lds, coarse, fine, j);

  // Hop 0 read the old tail above (and every thread has passed the
  // barriers inside the transform), so it can now store the new one.
  if (update_tail && h == 0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) tl[j + 256 * r] = ys[n_t - kHist + j + 256 * r];
  }

  float2 U[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) U[r] = v[r];
  // Chirp phase of bin q (signed q_s) for trial t, in cycles:
  //   frac(kappa T / (f_k + nu_q)) + q_s D / 4096
  //     = frac(A) - A g_q + (q_s mod 4) / 4   (mod 1),
  // with A = kappa T / f_k, g_q = x / (1 + x), x = nu_q / f_k from the plan
  // table, and q_s mod 4 = j mod 4 for every bin of thread j.  The residual
  // A g_q is below ~0.4 cycles; the hardware sine/cosine take revolutions.
  const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(gq), 0, n_sb * kNfft * 4, kRawBufferWord3);
  const float e = 0.25f * (float)(j & 3);
  const float scale = 1.0f / 4096.0f;
  for (int jt = 0; jt < n_tec; ++jt) {
    const int jo = opaque(j);
    const float bse = base[jt * n_sb + s] + e, A = afac[jt * n_sb + s];
    const int goff = 4 * (s * kNfft + jo);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float g = __uint_as_float(
          __builtin_amdgcn_raw_buffer_load_b32(grs, goff, 1024 * r, 0));
      float c = fmaf(-A, g, bse);
      c -= rintf(c);
      const float sn = __builtin_amdgcn_sinf(c), cs = __builtin_amdgcn_cosf(c);
      v[r] = cmul(U[r], make_float2(cs, -sn));
    }
    __syncthreads();  // previous trial's last LDS reads are done
    fft4096<true>(v, lds, coarse, fine, jo);
    float2 *out = d + (((long)b * n_tec + jt) * n_sb + s) * n_t + hs;
#pragma unroll
    for (int r = 8; r < 16; ++r)
      out[j + 256 * (r - 8)] = make_float2(v[r].x * scale, v[r].y * scale);
  }
}

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_dedisperse(lp_ctx *ctx, const lp_band *band,
                                   const double *tec_tecu, int32_t n_tec,
                                   const void *y, int32_t n_beams,
                                   int64_t n_t, void *tail, int32_t flags,
                                   void *d, void *hip_stream) {
  if (!ctx || !tec_tecu || !y || !tail || !d)
    return set_error(LP_EINVAL, "lp_dedisperse: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (n_tec <= 0 || n_tec > 4096)
    return set_error(LP_EINVAL, "lp_dedisperse: n_tec %d", n_tec);
  for (int j = 0; j < n_tec; ++j)
    if (!(tec_tecu[j] >= 0.0 && tec_tecu[j] <= 1000.0))
      return set_error(LP_EINVAL, "lp_dedisperse: TEC %g outside [0, 1000]",
                       tec_tecu[j]);
  if (n_beams <= 0)
    return set_error(LP_EINVAL, "lp_dedisperse: n_beams %d", n_beams);
  if (n_t <= 0 || n_t % kHop != 0)
    return set_error(LP_EINVAL,
                     "lp_dedisperse: n_t %lld not a positive multiple of %d",
                     (long long)n_t, kHop);
  if (flags & ~LP_DD_KEEP_TAIL)
    return set_error(LP_EINVAL, "lp_dedisperse: unknown flags 0x%x", flags);
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<DdPlan> p;
  if ((rc = get_dd_plan(ctx, band, tec_tecu, n_tec, st, p))) return rc;
  return dd_launch(ctx, p.get(), band->n_sb, y, n_beams, n_t, tail,
                   !(flags & LP_DD_KEEP_TAIL), d, st);
}

namespace lp {
lp_status dd_launch(lp_ctx *ctx, DdPlan *p, int n_sb, const void *y,
                    int n_beams, long n_t, void *tail, bool update_tail,
                    void *d, hipStream_t st) {
  lp_status rc;
  if ((rc = plan_wait(p, st))) return rc;
  const int n_hop = (int)(n_t / kHop);
  const long nb = (long)n_beams * n_sb * n_hop;
  if (nb > 0x7fffffffL)
    return set_error(LP_EINVAL, "lp_dedisperse: grid too large");
  hipLaunchKernelGGL(dd_kernel, dim3((unsigned)nb), dim3(kDdThreads), 0, st,
                     static_cast<const float2 *>(y), static_cast<float2 *>(tail),
                     update_tail ? 1 : 0, static_cast<float2 *>(d),
                     ctx->tw4096.as<const float2>(), p->base.as<const float>(),
                     p->afac.as<const float>(), p->gq.as<const float>(), n_sb,
                     p->n_tec, n_t, n_hop, nb);
  LP_HIP(hipGetLastError());
  return LP_OK;
}
}  // namespace lp

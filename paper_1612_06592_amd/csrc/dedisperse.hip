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
// two exchanges through a padded 34 KB LDS tile.  Each thread's base
// twiddle of a pass comes from two small LDS tables and its powers from a
// product tree (tables of all powers were measured slower: this kernel is
// close to bound by LDS instructions as well as VALU).  The forward
// spectrum stays in registers across all trials.  A trial's chirp phase is
// formed per bin from FP64-reduced constants and taken through the
// hardware sine and cosine; on a uniform grid only the first trial's is,
// and trial t + 1's chirp is trial t's times a per-bin factor read from a
// table formed in FP64 (a table of every trial's factors, one complex load
// per bin and trial instead of the phase, made the single-trial workloads
// slower: C3 2.70 -> 2.79 ms).
#include <cmath>

#include "fft_dev.h"
#include "lp_internal.h"

namespace lp {

constexpr int kDdThreads = 256;
constexpr int kDdLds = 4096 + 128;  // slot of element 4095 is 4222

// 16-point DFT returning only outputs 8..15 (in v[8..15]; v[0..7] are left
// undefined): the second radix-4 stage forms just its outputs 2 and 3.
template <bool INV>
__device__ __forceinline__ void dft16_hi(float2 *v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
      v[n2 + 4 * k1] = tw16<INV>(v[n2 + 4 * k1], n2 * k1);
  }
  float2 o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    const float2 a = v[4 * k1], b = v[4 * k1 + 1], c = v[4 * k1 + 2],
                 d = v[4 * k1 + 3];
    const float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d),
                 t3 = csub(b, d);
    o[k1] = csub(t0, t2);  // output k1 + 8
    // output k1 + 12: t1 + i t3 (forward) or t1 - i t3 (inverse)
    o[4 + k1] = INV ? make_float2(t1.x + t3.y, t1.y - t3.x)
                    : make_float2(t1.x - t3.y, t1.y + t3.x);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) v[8 + i] = o[i];
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

// LDS twiddle tables of one workgroup (w = exp(-2 pi i / 4096)):
//   coarse[c] = w^(16 c) (c < 256), fine[f] = w^f (f < 16).
struct DdTw {
  float2 coarse[256];
  float2 fine[16];
};

// 4096-point transform of v[r] = in[j + 256 r] (j = thread); on return
// v[r] = out[j + 256 r] (HI: only r >= 8).  Unnormalised; INV selects
// exp(+2 pi i ...).
template <bool INV, bool HI>
__device__ __forceinline__ void fft4096(float2 *v, float2 *lds,
                                        const DdTw &tw, int j) {
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
  // Pass 1 (Ns = 16): twiddle w^(16 (j mod 16) r).
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[sj + 264 * r];
  {
    const float2 w = tw.coarse[j & 15];
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
  // Pass 2 (Ns = 256): twiddle w^(j r); output index j + 256 r stays in
  // registers.
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[sj + 264 * r];
  {
    const float2 w = cmul(tw.coarse[j >> 4], tw.fine[j & 15]);
    pow16_twiddle(v, INV ? make_float2(w.x, -w.y) : w);
  }
  if (HI)
    dft16_hi<INV>(v);
  else
    dft16<INV>(v);
}

// Chirp factor exp(-2 pi i c) for a phase c in cycles, |c| <= 1/2 after the
// reduction; the hardware sine and cosine take revolutions.
__device__ __forceinline__ float2 chirp(float c) {
  c -= rintf(c);
  return make_float2(__builtin_amdgcn_cosf(c), -__builtin_amdgcn_sinf(c));
}

// REC: the trials are uniformly spaced, so the first trial's chirp comes
// from its phase and each next one is the previous one times
// rstep[s][q] (float2 [S][N_fft]).
template <bool REC>
__global__ __launch_bounds__(kDdThreads)
__attribute__((amdgpu_waves_per_eu(4, 8))) void dd_kernel(
    const float2 *__restrict__ y, float2 *__restrict__ tail, int update_tail,
    float2 *__restrict__ d, const float2 *__restrict__ tw,
    const float *__restrict__ base, const float *__restrict__ afac,
    const float2 *__restrict__ rstep, const float *__restrict__ gq, int n_sb,
    int n_tec, long n_t, int n_hop, long n_blocks) {
  __shared__ float2 lds[kDdLds];
  __shared__ DdTw tws;
  {
    const int i = threadIdx.x;  // tw[n] = w^n, n < 4096
    tws.coarse[i] = tw[16 * i];
    if (i < 16) tws.fine[i] = tw[i];
  }
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

  fft4096<false, false>(v, lds, tws, j);

  // Hop 0 read the old tail above (and every thread has passed the
  // barriers inside the transform), so it can now store the new one.
  if (update_tail && h == 0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) tl[j + 256 * r] = ys[n_t - kHist + j + 256 * r];
  }

  // The inverse transform's 1 / 4096 applied to the spectrum (a power of
  // two: exact, so every later rounding is the same as scaling the output).
  float2 U[16];
#pragma unroll
  for (int r = 0; r < 16; ++r)
    U[r] = make_float2(v[r].x * (1.0f / 4096.0f), v[r].y * (1.0f / 4096.0f));
  // Chirp phase of bin q (signed q_s) for trial t, in cycles:
  //   frac(kappa T / (f_k + nu_q)) + q_s D / 4096
  //     = frac(A) - A g_q + (q_s mod 4) / 4   (mod 1),
  // with A = kappa T / f_k, g_q = x / (1 + x), x = nu_q / f_k from the plan
  // table, and q_s mod 4 = j mod 4 for every bin of thread j.  The residual
  // A g_q is below ~0.4 cycles.
  const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(gq), 0, n_sb * kNfft * 4, kRawBufferWord3);
  const float e = 0.25f * (float)(j & 3);
  float2 *outb = d + ((long)b * n_tec * n_sb + s) * n_t + hs + j;
  const long trial_stride = (long)n_sb * n_t;
  if (REC) {
    // U becomes the first trial's chirped spectrum; R the per-trial factor.
    const float bse = base[s] + e, A = afac[s];
    const float2 *rs = rstep + s * kNfft + j;
    float2 R[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float g = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          grs, 4 * (s * kNfft + j), 1024 * r, 0));
      U[r] = cmul(U[r], chirp(fmaf(-A, g, bse)));
      R[r] = rs[256 * r];
    }
    for (int jt = 0; jt < n_tec; ++jt) {
      const int jo = opaque(j);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        v[r] = U[r];
        U[r] = cmul(U[r], R[r]);
      }
      __syncthreads();  // previous trial's last LDS reads are done
      fft4096<true, true>(v, lds, tws, jo);
      float2 *out = outb + jt * trial_stride;
#pragma unroll
      for (int r = 8; r < 16; ++r) out[256 * (r - 8)] = v[r];
    }
  } else {
    for (int jt = 0; jt < n_tec; ++jt) {
      const int jo = opaque(j);
      const float bse = base[jt * n_sb + s] + e, A = afac[jt * n_sb + s];
      const int goff = 4 * (s * kNfft + jo);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float g = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(grs, goff, 1024 * r, 0));
        v[r] = cmul(U[r], chirp(fmaf(-A, g, bse)));
      }
      __syncthreads();  // previous trial's last LDS reads are done
      fft4096<true, true>(v, lds, tws, jo);
      float2 *out = outb + jt * trial_stride;
#pragma unroll
      for (int r = 8; r < 16; ++r) out[256 * (r - 8)] = v[r];
    }
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
                   !(flags & LP_DD_KEEP_TAIL), d, 0, n_tec, st);
}

namespace lp {
lp_status dd_launch(lp_ctx *ctx, DdPlan *p, int n_sb, const void *y,
                    int n_beams, long n_t, void *tail, bool update_tail,
                    void *d, int j0, int nj, hipStream_t st) {
  lp_status rc;
  if ((rc = plan_wait(p, st))) return rc;
  const int n_hop = (int)(n_t / kHop);
  const long nb = (long)n_beams * n_sb * n_hop;
  if (nb > 0x7fffffffL)
    return set_error(LP_EINVAL, "lp_dedisperse: grid too large");
  if (j0 < 0 || nj <= 0 || j0 + nj > p->n_tec)
    return set_error(LP_EINVAL, "de-dispersion: trials %d..%d of %d", j0,
                     j0 + nj - 1, p->n_tec);
  const size_t jo = (size_t)j0 * n_sb;
  auto kern = p->uniform && nj >= 2 ? dd_kernel<true> : dd_kernel<false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kDdThreads), 0, st,
                     static_cast<const float2 *>(y), static_cast<float2 *>(tail),
                     update_tail ? 1 : 0, static_cast<float2 *>(d),
                     ctx->tw4096.as<const float2>(),
                     p->base.as<const float>() + jo,
                     p->afac.as<const float>() + jo,
                     p->rstep.as<const float2>(),
                     p->gq.as<const float>(), n_sb, nj, n_t, n_hop, nb);
  LP_HIP(hipGetLastError());
  return LP_OK;
}
}  // namespace lp

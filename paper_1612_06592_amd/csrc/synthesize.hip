// Time-domain synthesis from the polyphase-filtered subbands (Winchen et
// al. 2016, Sec. 2 and Sec. 3: the PPF inversion that recovers the 5 ns
// signal), fused with the Hilbert envelope used by the trigger.
//
// Per series (beam, trial) and frame m:
//   Z_m[n] = sum_k d_k[m] exp(+2 pi i k n / 1024)        (1024-point IFFT)
//   z[1024 m + n] = sum_{t<16} g[1024 t + n] Z_{m-t}[n]   (polyphase FIR)
// with g = M h.  Only positive bins are filled, so z is analytic: the real
// series is 2 Re z and the envelope |2 z|.  The kernel takes the taps as
// 2 g, so its sums are 2 z directly (scaling by 2 is exact).
//
// One 1024-thread workgroup per (series, block of F frames).  Frames are
// transformed 16 at a time in a 139 KB LDS tile (radix 16, 16, 4 Stockham
// passes): wave w transforms frame w of each chunk on its own, so the
// exchanges between passes stay inside the wave (through LDS after pass 0,
// by lane swaps across rows of 16 after pass 1) and a chunk needs two
// workgroup barriers (transforms done; FIR done).  Thread n then owns FIR
// column n and keeps
// Z_{m-15..m}[n] and its 16 taps in registers, so each output sample costs
// 16 complex-by-real FMAs and nothing is written to HBM except the
// per-frame envelope maximum (+ arg), per-16-frame sums of (2 Re z)^2 and,
// on request, the real series.
#include <cmath>

#include "fft_dev.h"
#include "lp_internal.h"

namespace lp {

constexpr int kSynThreads = 1024;

constexpr int kSynFs = 1089;  // LDS frame stride (>= pad16(1023)+1, odd)

struct SynCand {
  float emax;
  int arg;
};

// Wavefront reductions by DPP lane exchanges (no LDS, no address
// arithmetic).  Steps: quad lanes 1 and 2 apart, then the mirrors of each
// 8 and 16 lanes, after which every lane holds its 16-lane row's result;
// then lane 15 of rows 0 and 2 into rows 1 and 3, and lane 31 into rows 2
// and 3, so lane 63 holds the wavefront's result.
constexpr int kDppQuadX1 = 0xB1, kDppQuadX2 = 0x4E, kDppHalfMirror = 0x141,
              kDppMirror = 0x140, kDppBcast15 = 0x142, kDppBcast31 = 0x143;

// Lane exchange CTRL in the rows of ROWS; lanes of the other rows get
// `old`.  (Every exchange here reads lanes inside the wavefront.)
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int v, int old) {
  if constexpr (ROWS == 0xF)
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
  else
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v, float old) {
  return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(v), __float_as_int(old)));
}

// Sum over the wavefront, valid in lane 63.
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_f<kDppQuadX1, 0xF>(v, 0.f);
  v += dpp_f<kDppQuadX2, 0xF>(v, 0.f);
  v += dpp_f<kDppHalfMirror, 0xF>(v, 0.f);
  v += dpp_f<kDppMirror, 0xF>(v, 0.f);
  v += dpp_f<kDppBcast15, 0xA>(v, 0.f);
  v += dpp_f<kDppBcast31, 0xC>(v, 0.f);
  return v;
}

// Unsigned maximum over the wavefront, returned to every lane (rows
// outside the broadcast masks take the maximum with themselves).
__device__ __forceinline__ unsigned wave_umax_dpp(unsigned v) {
  v = max(v, (unsigned)dpp_i<kDppQuadX1, 0xF>((int)v, 0));
  v = max(v, (unsigned)dpp_i<kDppQuadX2, 0xF>((int)v, 0));
  v = max(v, (unsigned)dpp_i<kDppHalfMirror, 0xF>((int)v, 0));
  v = max(v, (unsigned)dpp_i<kDppMirror, 0xF>((int)v, 0));
  v = max(v, (unsigned)dpp_i<kDppBcast15, 0xA>((int)v, (int)v));
  v = max(v, (unsigned)dpp_i<kDppBcast31, 0xC>((int)v, (int)v));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// MASKED: some chunk straddles the end of the warm-up (`warm` - frame0 not
// a multiple of 16), so the statistics mask frame by frame; otherwise a
// chunk is either all warm-up or all valid.  NR: bins j + 64 r with r >= NR
// are empty in the band (its highest bin is below 64 NR), so the first
// transform pass reads NR inputs and the rest are known zeros.
template <bool MASKED, int NR>
__global__ __launch_bounds__(kSynThreads) void syn_kernel(
    const float2 *__restrict__ d, float2 *__restrict__ hist,
    const short *__restrict__ binmap, const float *__restrict__ taps,
    const float2 *__restrict__ tw, float *__restrict__ x_out,
    SynCand *__restrict__ cand, float *__restrict__ psum, int n_sb, long n_t,
    long frame0, long warm, long per_wg, long total, long cand_nt,
    long cand_t0) {
  __shared__ float2 lds[16 * kSynFs];
  // Base twiddles of the two twiddled passes; each lane forms the powers it
  // needs by products (reading every power from LDS tables was 4 % slower:
  // the transform is bound by the latency of its LDS accesses):
  //   tw_p1[a] = exp(+2 pi i 4 a / 1024)   (pass 1, a = j mod 16)
  //   tw_p2[t] = exp(+2 pi i t / 1024)     (pass 2, t < 256)
  __shared__ float2 tw_p1[16];
  __shared__ float2 tw_p2[256];
  __shared__ float red_s[16];
  // Byte offset in the series of the row of bin j + 64 r (lane j), or the
  // series size for an empty bin (a raw buffer load past the end reads 0).
  __shared__ unsigned roff_s[8 * 64];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int n = tid;  // FIR column

  float2 win[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) win[t] = make_float2(0.f, 0.f);
  if (tid < 256 + 16) {
    // From the table exp(-2 pi i n / 4096), conjugated.
    const int t = tid < 256 ? tid : 4 * (tid - 256);
    const float2 w = tw[4 * t];
    (tid < 256 ? tw_p2[tid] : tw_p1[tid - 256]) = make_float2(w.x, -w.y);
  }
  // Wave w transforms frame w of each 16-frame chunk; lane j is pass-0
  // butterfly j, reading bins j + 64 r (r < NR) at the offsets in roff_s.
  const unsigned ser_bytes = (unsigned)n_sb * (unsigned)n_t * 8u;
  if (tid < NR * 64) {
    const int si = binmap[tid];
    roff_s[tid] = si >= 0 ? (unsigned)si * (unsigned)n_t * 8u : ser_bytes;
  }
  __syncthreads();

  // This workgroup's frames: [g, g_end) of the series-major frame index
  // series * n_t + m, as segments of one series each (every segment starts
  // with its own 16-frame warm-up chunk).
  long g = (long)blockIdx.x * per_wg;
  const long g_end = min(g + per_wg, total);
  for (; g < g_end;) {
    const int series = (int)(g / n_t);
    const long m0 = g - (long)series * n_t;
    const long seg = min(g_end - g, n_t - m0);
    g += seg;
    const float2 *ds = d + (long)series * n_sb * n_t;
    float2 *hs = hist + (long)series * n_sb * kSynHist;
    const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float2 *>(ds), 0, (int)ser_bytes, kRawBufferWord3);
    const int n_chunk = (int)(seg / 16);
    float2 pre[NR];
    auto fetch = [&](long mc_) {
      const long m = mc_ + wave;
      if (m >= 0) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        const unsigned mo = (unsigned)m * 8u;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const u2 b = __builtin_amdgcn_raw_buffer_load_b64(
              drs, roff_s[64 * r + lane] + mo, 0, 0);
          pre[r] = make_float2(__uint_as_float(b.x), __uint_as_float(b.y));
        }
      } else {
        // Before the stream block (warm-up chunk of workgroup 0): history.
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int si = binmap[lane + 64 * r];
          pre[r] = si >= 0 ? hs[si * kSynHist + (kSynHist + m)]
                           : make_float2(0.f, 0.f);
        }
      }
    };
    fetch(m0 - 16);
    for (int c = -1; c < n_chunk; ++c) {
      const long mc = m0 + 16L * c;  // first frame of the chunk
      const int no = opaque(n), lo = opaque(lane), wo = opaque(wave);
      float2 *fr = lds + wo * kSynFs;
      // ---- pass 0 (radix 16, Ns = 1) of frame wo: butterfly lo.  Every
      // exchange of this frame stays inside the wave, whose LDS operations
      // execute in issue order; the fences only keep the compiler from moving
      // reads above the writes they depend on.
      float2 v[16];
#pragma unroll
      for (int r = 0; r < NR; ++r) v[r] = pre[r];
#pragma unroll
      for (int r = NR; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
      dft16<true, NR>(v);
      // pad16(16 j + r) = 17 j + r.
#pragma unroll
      for (int r = 0; r < 16; ++r) fr[17 * lo + r] = v[r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      {
        // pad16(j + 64 r) = j + j / 16 + 68 r for j < 64.
        const int b1 = lo + (lo >> 4);
        // ---- pass 1 (radix 16, Ns = 16).
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = fr[b1 + 68 * r];
        {
          // v[r] *= w^r, w = exp(2 pi i (j mod 16) / 256): a product tree
          // of depth 4, each power used as soon as it exists.
          const float2 w1 = tw_p1[lo & 15];
          const float2 w2 = cmul(w1, w1), w4 = cmul(w2, w2), w8 = cmul(w4, w4);
          const float2 w3 = cmul(w2, w1), w7 = cmul(w4, w3);
          v[1] = cmul(v[1], w1);
          v[2] = cmul(v[2], w2);
          v[3] = cmul(v[3], w3);
          v[4] = cmul(v[4], w4);
          v[5] = cmul(v[5], cmul(w4, w1));
          v[6] = cmul(v[6], cmul(w4, w2));
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
        dft16<true>(v);
        pass2_gather(v);  // v[4 q + m] = element j + 64 q + 256 m
        // ---- pass 2 (radix 4, Ns = 256): butterflies j + 64 q, q < 4,
        // written to their output slots
        // pad16(j + 64 q + 256 k) = j + j / 16 + 68 q + 272 k (j < 64).
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int jt = lo + 64 * q;
          float2 *sl = fr + b1 + 68 * q;
          float2 a0 = v[4 * q], a1 = v[4 * q + 1], a2 = v[4 * q + 2],
                 a3 = v[4 * q + 3];
          const float2 u1 = tw_p2[jt], u2 = cmul(u1, u1), u3 = cmul(u2, u1);
          a1 = cmul(a1, u1);
          a2 = cmul(a2, u2);
          a3 = cmul(a3, u3);
          dft4<true>(a0, a1, a2, a3);
          sl[0] = a0;
          sl[272] = a1;
          sl[544] = a2;
          sl[816] = a3;
        }
      }
      // Taps (2 g) of column n, in flight across the barrier.  A raw buffer
      // view of the 16 x 1024 taps: tap t of column n is at the constant
      // offset 4096 t plus 4 n.
      const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(taps), 0, 16 * 1024 * 4, kRawBufferWord3);
      float g[16];
#pragma unroll
      for (int t = 0; t < 16; ++t)
        g[t] = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(trs, 4 * no, 4096 * t, 0));
      __syncthreads();  // every frame of the chunk is transformed
      if (c == -1 && m0 == 0) {
        // Every history read of this block happened above: store the new
        // history, the last 16 frames of d.
        for (int i = tid; i < n_sb * kSynHist; i += kSynThreads) {
          int si = i / kSynHist, fi = i % kSynHist;
          hs[i] = ds[(long)si * n_t + (n_t - kSynHist + fi)];
        }
      }
      // Next chunk's inputs are in flight while this chunk is filtered.
      if (c + 1 < n_chunk) fetch(mc + 16);
      // ---- FIR, envelope, statistics for the 16 frames of this chunk.
      if (c < 0) {
#pragma unroll
        for (int fi = 0; fi < 16; ++fi) win[fi] = lds[fi * kSynFs + pad16(no)];
        __syncthreads();  // reads done before the next chunk's transforms
        continue;
      }
      float acc_s = 0.f;
      // Frames before `warm` (stream time) stay out of the statistics.
      const long fv = warm - (frame0 + mc);
      const int first_valid = fv <= 0 ? 0 : (fv >= 16 ? 16 : (int)fv);
      float *xo = x_out ? x_out + ((long)series * n_t + mc) * 1024 + no : nullptr;
      // (zr, zi) = 2 z of frame fi: 2 Re z is the real series, |2 z|^2 the
      // squared envelope; the slot is consumed, so it takes the latter, in
      // its x word for columns with bit 4 clear and its y word otherwise (the
      // 16-column groups then alternate between even and odd banks).
      const int ecomp = (no >> 4) & 1;
#pragma unroll
      for (int fi = 0; fi < 16; ++fi) {
        float2 *slot = lds + fi * kSynFs + pad16(no);
        win[fi] = *slot;
        float zr = 0.f, zi = 0.f;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          float2 w = win[(fi - t) & 15];
          zr = fmaf(g[t], w.x, zr);
          zi = fmaf(g[t], w.y, zi);
        }
        if (!MASKED || fi >= first_valid) acc_s = fmaf(zr, zr, acc_s);
        if (xo) xo[(long)fi * 1024] = zr;
        reinterpret_cast<float *>(slot)[ecomp] = zr * zr + zi * zi;
      }
      if (!MASKED && first_valid != 0) acc_s = 0.f;  // first_valid is 16
      acc_s = wave_sum_dpp(acc_s);
      if (lo == 63) red_s[wo] = acc_s;
      __syncthreads();
      // Wave w finds the envelope maximum of frame w and its lowest n: the
      // maximum first, then per row n = 64 i + lane a ballot of the lanes
      // holding it; the first row with a hit and its lowest lane give n.
      // Squared envelopes are >= +0, so their bit patterns order as unsigned
      // integers: the maximum is an exact selection.
      {
        // Lane l holds n = l + 64 i at slot pad16(n) = l + l / 16 + 68 i,
        // envelope word (n / 16) mod 2 = (l / 16) mod 2.
        const float *fl = reinterpret_cast<const float *>(
                              lds + wo * kSynFs + lo + (lo >> 4)) +
                          ((lo >> 4) & 1);
        unsigned e2[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) e2[i] = __float_as_uint(fl[2 * 68 * i]);
        unsigned bv = e2[0];
#pragma unroll
        for (int i = 1; i < 16; ++i) bv = max(bv, e2[i]);
        bv = wave_umax_dpp(bv);
        int bi = 0;
#pragma unroll
        for (int i = 15; i >= 0; --i) {
          const unsigned long long hit = __builtin_amdgcn_ballot_w64(e2[i] == bv);
          if (hit) bi = 64 * i + __builtin_ctzll(hit);
        }
        if (lo == 0) {
          SynCand o;
          o.emax = sqrtf(__uint_as_float(bv));
          o.arg = bi;
          cand[(long)series * cand_nt + cand_t0 + mc + wo] = o;
        }
      }
      if (tid == 64) {
        float sum = 0.f;
        for (int w = 0; w < 16; ++w) sum += red_s[w];
        psum[(long)series * (cand_nt / 16) + (cand_t0 + mc) / 16] = sum;
      }
    }
  }  // segments
}

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_synthesize(lp_ctx *ctx, const lp_band *band,
                                   const void *d, int32_t n_series,
                                   int64_t n_t, int64_t frame0, void *hist,
                                   float *x_out, void *cand,
                                   void *hip_stream) {
  if (!ctx || !d || !hist || !cand)
    return set_error(LP_EINVAL, "lp_synthesize: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (n_series <= 0 || n_series > 65535)
    return set_error(LP_EINVAL, "lp_synthesize: n_series %d", n_series);
  if (n_t <= 0 || n_t % kHop != 0)
    return set_error(LP_EINVAL,
                     "lp_synthesize: n_t %lld not a positive multiple of %d",
                     (long long)n_t, kHop);
  if (frame0 < 0) return set_error(LP_EINVAL, "lp_synthesize: frame0 < 0");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<SynPlan> p;
  if ((rc = get_syn_plan(ctx, band, st, p))) return rc;
  return syn_launch(ctx, p.get(), band->n_sb, d, n_series, n_t, frame0, hist,
                    x_out, cand, n_t, 0, 0, n_series, st);
}

namespace lp {
lp_status syn_launch(lp_ctx *ctx, SynPlan *p, int n_sb, const void *d,
                     int n_series, long n_t, long frame0, void *hist,
                     float *x_out, void *cand, long cand_nt, long cand_t0,
                     int series0, int n_series_total, hipStream_t st) {
  lp_status rc;
  if ((rc = plan_wait(p, st))) return rc;
  // The kernel addresses one series' subbands with 32-bit byte offsets
  // (empty bins at one row past the end).
  if ((long)(n_sb + 1) * n_t * 8 >= (1L << 32))
    return set_error(LP_EINVAL, "synthesis: %d subbands x %ld frames too large",
                     n_sb, n_t);
  // Frames per workgroup: each workgroup is one CU's tile for its life and
  // walks a contiguous range of the series-major frame index, paying a
  // 16-frame warm-up chunk for every series its range touches.  Candidates:
  // the old lengths that divide n_t (ranges inside one series) and ranges
  // of total / (k CUs) frames (k = 1, 2, 4, 8 rounds of workgroups); each
  // scored by the frames filtered over the longest workgroup's work times
  // the rounds (the longest range on ties).
  const long total = (long)n_series * n_t;
  long per_wg = 16;
  double best = -1.0;
  auto consider = [&](long f) {
    if (f <= 0) return;
    const long nw = (total + f - 1) / f;
    const long rounds = (nw + ctx->n_cu - 1) / ctx->n_cu;
    const long segs = (f % n_t == 0 || n_t % f == 0) ? (f + n_t - 1) / n_t
                                                     : (f + n_t - 1) / n_t + 1;
    const double eff =
        (double)total / ((double)rounds * ctx->n_cu * (f + 16.0 * segs));
    if (eff > best + 1e-12 || (eff > best - 1e-12 && f > per_wg)) {
      best = eff;
      per_wg = f;
    }
  };
  for (int f : {2048, 1024, 512, 256, 128, 64, 32, 16})
    if (n_t % f == 0) consider(f);
  for (int k : {1, 2, 4, 8}) {
    const long slots = (long)k * ctx->n_cu;
    consider(((total + slots - 1) / slots + 15) / 16 * 16);
  }
  const long n_wg = (total + per_wg - 1) / per_wg;
  if (n_wg > 0x7fffffffL)
    return set_error(LP_EINVAL, "synthesis: grid too large");
  const long warm = kDelay + kTaps;
  const bool masked = frame0 < warm && (warm - frame0) % 16 != 0;
  char *cb = static_cast<char *>(cand);
  SynCand *cd = reinterpret_cast<SynCand *>(cb) + (size_t)series0 * cand_nt;
  float *ps = reinterpret_cast<float *>(cb + (size_t)n_series_total * cand_nt * 8) +
              (size_t)series0 * (cand_nt / 16);
  // Kernel for the band's highest bin: pass-0 rows 4, 5, 6 or 8.
  decltype(&syn_kernel<false, 8>) kern;
  if (p->kmax < 256)
    kern = masked ? syn_kernel<true, 4> : syn_kernel<false, 4>;
  else if (p->kmax < 320)
    kern = masked ? syn_kernel<true, 5> : syn_kernel<false, 5>;
  else if (p->kmax < 384)
    kern = masked ? syn_kernel<true, 6> : syn_kernel<false, 6>;
  else
    kern = masked ? syn_kernel<true, 8> : syn_kernel<false, 8>;
  hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(kSynThreads), 0, st,
                     static_cast<const float2 *>(d),
                     static_cast<float2 *>(hist), p->binmap.as<const short>(),
                     p->taps2.as<const float>(), ctx->tw4096.as<const float2>(),
                     x_out, cd, ps, n_sb, n_t, frame0, warm, per_wg, total,
                     cand_nt, cand_t0);
  LP_HIP(hipGetLastError());
  return LP_OK;
}
}  // namespace lp

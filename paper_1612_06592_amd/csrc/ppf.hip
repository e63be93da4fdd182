// Inversion of the polyphase filterbank (Winchen et al. 2016, Sec. 3: the
// 5 ns signal is recovered by solving the sparse system H x = y for the
// filtered subband data y with LSMR; about 25 iterations converge), with
// LSMR as published by Fong & Saunders (SIAM J. Sci. Comput. 33, 2011,
// Algorithm 1, no damping, x_0 = 0).
//
// H is the analysis filterbank restricted to the recorded channels k[s]:
//   v_m[r]  = sum_{t<16} h[1024 t + r] x[1024 (m - t) + 1023 - r]
//   y_s[m]  = sum_{r<1024} v_m[r] exp(+2 pi i k[s] r / 1024)
// for output frames m < n_frames of a real series x of F = n_frames - 15
// frames (zero outside).  Its real adjoint is
//   W_m[r]  = Re sum_s y_s[m] exp(-2 pi i k[s] r / 1024)
//   (H^T y)[1024 j + 1023 - r] = sum_{t<16} h[1024 t + r] W_{j + t}[r].
//
// Kernels.  Both operators stream 256 frames per 1024-thread workgroup in
// chunks of 32 real frames, packed two per complex 1024-point transform
// (16 transforms per chunk in a 139 KB LDS tile, Stockham radix 16, 16,
// 4, wave w transforming packed frame w).  Thread r owns FIR column r and
// keeps 16 frames of it in registers.  A series' arrays are addressed with
// 32-bit offsets (n_frames <= 2^19).
//   ppf_fwd_kernel: FIR (16 FMA per sample) -> packed transform -> the
//     recorded bins of both frames from bins k and 1024 - k.  In LSMR mode
//     it also forms u = H v - (alpha / beta) u_old with its squared-norm
//     partial sums, and applies the previous iteration's elementwise
//     update of hbar, x and h while it reads v.
//   ppf_adj_kernel: the recorded bins of two frames -> one packed
//     Hermitian spectrum -> transform -> anti-causal FIR.  In LSMR mode
//     it forms p = H^T u - (beta / alpha) p_old and its norm partials.
// LSMR's scalar recurrences (rotations P_k and Pbar_k) run in FP64 in
// one-wave kernels between the operator launches, on the same stream, so
// a solve needs no host synchronisation.  Vectors are FP32 in HBM.
#include <cmath>

#include "fft_dev.h"
#include "lp_internal.h"

namespace lp {

constexpr int kPpfThreads = 1024;
constexpr int kPpfFs = 1090;       // LDS stride of one packed frame (float2)
constexpr int kPpfWg = 256;        // frames per workgroup
constexpr int kPpfChunk = 32;      // real frames per chunk
constexpr int kPpfNormParts = 2048; // partial sums of ||y||^2 per series
constexpr int kPpfStateBytes = 128;
// Frames per series of the operators: with nf <= 2^19 every byte offset
// into one series' arrays (and into its n_sb <= 511 rows of nf complex
// frames, chunk overrun included) stays below 2^31.
constexpr long kPpfMaxFrames = 1L << 19;

enum { kFwdAnalyze = 0, kFwdLsmr = 1, kFwdResid = 2, kFwdStation = 3 };
enum { kAdjPlain = 0, kAdjLsmr = 1 };

// LSMR state of one series (device memory, written by the scalar kernels).
struct LsmrState {
  double alpha, beta, alphabar, zetabar, rho, rhobar, cbar, sbar;
  float p_scale;  // v_k = p * p_scale            (1 / alpha_k)
  float q_scale;  // u_new = H v - q_scale * q    (alpha_k / beta_k)
  float u_scale;  // u = q * u_scale              (1 / beta_{k+1})
  float v_scale;  // p_new = H^T u - v_scale * p  (beta_{k+1} / alpha_k)
  float c_hbar, c_x, c_h;  // pending elementwise update
  int first;      // no update yet: h = v, hbar = x = 0
  int done;       // the bidiagonalisation ended (alpha or beta zero)
};
static_assert(sizeof(LsmrState) <= kPpfStateBytes, "state size");

// Twiddle tables of the wave-local transform (filled once per workgroup
// from the table exp(-2 pi i n / 4096), conjugated; every angle index is
// below 1024):
//   tw_p1[a][r] = exp(+2 pi i 4 a r / 1024), rows of 17 entries so the 16
//                 rows one wave reads fall on distinct banks;
//   tw_p2[q][t] = exp(+2 pi i (q + 1) t / 1024), t < 256.
constexpr int kTwP1 = 16 * 17, kTwP2 = 3 * 256;
__device__ __forceinline__ void fill_tw_tables(const float2 *tw,
                                               float2 *tw_p1, float2 *tw_p2) {
  const int tid = threadIdx.x;
  int idx;
  float2 *dst;
  if (tid < 256) {
    idx = 4 * (tid >> 4) * (tid & 15);
    dst = tw_p1 + (tid >> 4) * 17 + (tid & 15);
  } else {
    const int e = tid - 256;
    idx = (e / 256 + 1) * (e % 256);
    dst = tw_p2 + e;
  }
  const float2 w = tw[4 * idx];
  *dst = make_float2(w.x, -w.y);
}

// A wavefront-scope fence: the wave's LDS operations execute in order, so
// this only keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The 1024-point Stockham transform (radix 16, 16, 4) of LDS frame fr by
// one wave, lane j = butterfly: PASS0 also runs pass 0 on the frame in
// natural order; otherwise pass 0's output is already in place.  No
// workgroup barrier: the caller orders the frame's producers before and
// its consumers after.  Pass 1 hands its output to pass 2 in registers
// (pass2_gather).  Slots in closed form (j < 64):
//   pad16(j + 64 r) = j + j / 16 + 68 r,   pad16(16 j + r) = 17 j + r.
template <bool INV, bool PASS0>
__device__ __forceinline__ void fft1024_wave(float2 *fr, const float2 *tw_p1,
                                             const float2 *tw_p2, int j) {
  const int b1 = j + (j >> 4);
  float2 v[16];
  if constexpr (PASS0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = fr[b1 + 68 * r];
    dft16<INV>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) fr[17 * j + r] = v[r];
    wave_lds_fence();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = fr[b1 + 68 * r];
  {
    const float2 *twr = tw_p1 + (j & 15) * 17;  // 2 pi (j mod 16) r / 256
#pragma unroll
    for (int r = 1; r < 16; ++r)
      v[r] = INV ? cmul(v[r], twr[r]) : cmulc(v[r], twr[r]);
  }
  dft16<INV>(v);
  pass2_gather(v);  // v[4 q + m] = element j + 64 q + 256 m
  // Pass 2 writes each butterfly's outputs to the slots of its inputs,
  // pad16(j + 64 q + 256 k): the slots this lane read in pass 1.
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int jt = j + 64 * q;
    float2 *sl = fr + b1 + 68 * q;
    float2 a0 = v[4 * q], a1 = v[4 * q + 1], a2 = v[4 * q + 2],
           a3 = v[4 * q + 3];
    const float2 w1 = tw_p2[jt], w2 = tw_p2[256 + jt], w3 = tw_p2[512 + jt];
    if (INV) {
      a1 = cmul(a1, w1);
      a2 = cmul(a2, w2);
      a3 = cmul(a3, w3);
    } else {
      a1 = cmulc(a1, w1);
      a2 = cmulc(a2, w2);
      a3 = cmulc(a3, w3);
    }
    dft4<INV>(a0, a1, a2, a3);
    sl[0] = a0;
    sl[272] = a1;
    sl[544] = a2;
    sl[816] = a3;
  }
}

// Sum of one value per thread of a 1024-thread workgroup, fixed order;
// thread 0 stores it.
__device__ __forceinline__ void wg_sum_store(float acc, float *red,
                                             float *dst) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < kPpfThreads / 64; ++w) s += red[w];
    *dst = s;
  }
}

// H (kFwdAnalyze: yout = H x), one LSMR half-step (kFwdLsmr: q = H (p
// p_scale) - q_scale q in place, plus the pending update of hbar, x, h
// from p), the residual norm (kFwdResid: partials of |y - H x|^2), or the
// station filterbank (kFwdStation: int16 ADC input; the valid frames
// m' >= 15 of H, times oscale, rounded half to even and saturated to
// [-olim, olim - 1], go to sout [series][n_sb][nf - 30] as int16 pairs).
// xin is float, or int16 in station mode.
template <int MODE>
__global__ __launch_bounds__(kPpfThreads) void ppf_fwd_kernel(
    const void *__restrict__ xin_, const float2 *yin, float2 *yout,
    float *__restrict__ hv, float *__restrict__ hbar, float *__restrict__ xv,
    const LsmrState *__restrict__ st, float *__restrict__ part,
    const short *__restrict__ kbin, const float *__restrict__ taps,
    const float2 *__restrict__ tw, int n_sb, long nf, int n_part,
    float oscale = 1.f, int olim = 0, short2 *__restrict__ sout = nullptr) {
  __shared__ float2 lds[16 * kPpfFs];
  __shared__ float2 tw_p1[kTwP1], tw_p2[kTwP2];
  __shared__ float red[16];

  const int series = blockIdx.y;
  const long m0 = (long)blockIdx.x * kPpfWg;
  const long F = nf - (kTaps - 1);
  const long N = F * kM;
  const int tid = threadIdx.x;
  // Raw buffer views of this series' arrays, addressed by 32-bit byte
  // offsets (nf <= 2^19 keeps every offset below 2^31): a load past a
  // view's end, or at a negative offset (which wraps above 2^31), reads
  // zero and a store there is dropped - the zero frames before and after
  // the series.
  constexpr int xes = MODE == kFwdStation ? 2 : 4;  // input element bytes
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char *>(static_cast<const char *>(xin_)) + (long)series * N * xes,
      0, (int)(N * xes), kRawBufferWord3);
  auto ldx = [&](int e) -> float {  // input element e of the series
    if constexpr (MODE == kFwdStation)
      return (float)(short)__builtin_amdgcn_raw_buffer_load_b16(
          rx, (unsigned)e * xes, 0, 0);
    else
      return __uint_as_float(
          __builtin_amdgcn_raw_buffer_load_b32(rx, (unsigned)e * xes, 0, 0));
  };
  auto view = [&](float *a) {
    return __builtin_amdgcn_make_buffer_rsrc(a + (long)series * N, 0,
                                             (int)(N * 4), kRawBufferWord3);
  };
  const __amdgpu_buffer_rsrc_t rh = view(hv), rhb = view(hbar), rxv = view(xv);
  const long nout = nf - 2 * (kTaps - 1);  // station mode: valid frames
  const int ybytes = (int)((long)n_sb * nf * 8);
  const __amdgpu_buffer_rsrc_t ryi = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2 *>(yin) + (long)series * n_sb * nf, 0, ybytes,
      kRawBufferWord3);
  const __amdgpu_buffer_rsrc_t ryo = __builtin_amdgcn_make_buffer_rsrc(
      yout + (long)series * n_sb * nf, 0, ybytes, kRawBufferWord3);
  fill_tw_tables(tw, tw_p1, tw_p2);  // used after the first FIR barrier
  // Taps are g = 1024 h: fold 1 / 1024 into the input scale (exact).
  float ps = 1.f, qs = 0.f, c_hbar = 0.f, c_x = 0.f, c_h = 0.f;
  int first = 0;
  if (MODE == kFwdLsmr) {
    const LsmrState &S = st[series];
    ps = S.p_scale;
    qs = S.q_scale;
    c_hbar = S.c_hbar;
    c_x = S.c_x;
    c_h = S.c_h;
    first = S.first;
  }
  const float sc = ps * (1.f / 1024.f);

  // Ring of the last 16 input frames of column r (slot = frame mod 16).
  float ring[16];
  ring[0] = 0.f;
#pragma unroll
  for (int i = 1; i < 16; ++i)  // frames m0 - 15 .. m0 - 1 (zero if < 0)
    ring[i] = ldx((int)(m0 - 16 + i) * kM + (kM - 1 - tid)) * sc;
  float acc = 0.f;
  for (int c = 0; c < kPpfWg / kPpfChunk; ++c) {
    const long mc = m0 + (long)c * kPpfChunk;
    if (mc >= nf) break;
    const int ro = opaque(tid);
    const int lo = opaque(tid & 63), wo = opaque(tid >> 6);
    float g[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) g[t] = taps[t * kM + ro];
    __syncthreads();  // the previous chunk's reads of lds are done
    // ---- FIR of column r over the chunk's 32 frames, packed in pairs.
    // Element e0 + 1024 i is frame mc + i of column r (zero for frames
    // >= F: past the view).
    const int e0 = (int)mc * kM + (kM - 1 - ro);
    float prev = 0.f;
#pragma unroll
    for (int g8 = 0; g8 < 4; ++g8) {
      float pv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) pv[i] = ldx(e0 + (8 * g8 + i) * kM);
      if (MODE == kFwdLsmr) {
        // Pending update (hbar_k, x_k, h_{k+1}) on the unknowns this
        // workgroup owns, with v_{k+1} = p p_scale (frames >= F: the
        // stores fall past the views and are dropped).
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const unsigned o = (unsigned)(e0 + (8 * g8 + i) * kM) * 4u;
          const float v = pv[i] * ps;
          if (first) {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rh, o,
                                                  0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(0u, rhb, o, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(0u, rxv, o, 0, 0);
          } else {
            const float h0 = __uint_as_float(
                __builtin_amdgcn_raw_buffer_load_b32(rh, o, 0, 0));
            const float hb =
                h0 - c_hbar * __uint_as_float(
                                  __builtin_amdgcn_raw_buffer_load_b32(rhb, o, 0, 0));
            const float xn =
                __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rxv, o, 0, 0)) +
                c_x * hb;
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(hb), rhb, o,
                                                  0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(xn), rxv, o,
                                                  0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(
                __float_as_uint(v - c_h * h0), rh, o, 0, 0);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int fi = 8 * g8 + i;
        ring[fi & 15] = pv[i] * sc;
        float a = 0.f;
#pragma unroll
        for (int t = 0; t < 16; ++t) a = fmaf(g[t], ring[(fi - t) & 15], a);
        if (fi & 1)
          lds[(fi >> 1) * kPpfFs + pad16(ro)] = make_float2(prev, a);
        else
          prev = a;
      }
    }
    __syncthreads();
    // ---- Transform of the 16 packed frames v_e + i v_o: wave w transforms
    // packed frame w.
    fft1024_wave<true, true>(lds + wo * kPpfFs, tw_p1, tw_p2, lo);
    __syncthreads();
    // ---- Recorded bins of both frames of each pair:
    //   Y_even = (C_k + conj C_{M-k}) / 2,  Y_odd = (C_k - conj C_{M-k}) / 2i.
    for (int it = tid; it < 16 * n_sb; it += kPpfThreads) {
      const int s = it >> 4, pi = it & 15;
      const int k = kbin[s];
      const float2 *fr = lds + pi * kPpfFs;
      const float2 C = fr[pad16(k)], D = fr[pad16(kM - k)];
      float2 val[2];
      val[0] = make_float2(0.5f * (C.x + D.x), 0.5f * (C.y - D.y));
      val[1] = make_float2(0.5f * (C.y + D.y), -0.5f * (C.x - D.x));
      const long m = mc + 2 * pi;
      const unsigned ob = (unsigned)((int)s * (int)nf + (int)m) * 8u;
      auto ystore = [&](unsigned off, float2 w) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        u2 b = {__float_as_uint(w.x), __float_as_uint(w.y)};
        __builtin_amdgcn_raw_buffer_store_b64(b, ryo, off, 0, 0);
      };
      auto yload = [&](unsigned off) -> float2 {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        const u2 b = __builtin_amdgcn_raw_buffer_load_b64(ryi, off, 0, 0);
        return make_float2(__uint_as_float(b[0]), __uint_as_float(b[1]));
      };
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        if (m + e < nf) {
          if (MODE == kFwdAnalyze) {
            ystore(ob + 8 * e, val[e]);
          } else if (MODE == kFwdStation) {
            const long mo = m + e - (kTaps - 1);
            if (mo >= 0 && mo < nout) {
              const float lim = (float)olim;
              const float re = fminf(fmaxf(rintf(val[e].x * oscale), -lim),
                                     lim - 1.f);
              const float im = fminf(fmaxf(rintf(val[e].y * oscale), -lim),
                                     lim - 1.f);
              sout[((long)series * n_sb + s) * nout + mo] =
                  make_short2((short)re, (short)im);
            }
          } else if (MODE == kFwdLsmr) {
            const float2 q0 = yload(ob + 8 * e);
            const float2 qn = make_float2(val[e].x - qs * q0.x,
                                          val[e].y - qs * q0.y);
            ystore(ob + 8 * e, qn);
            acc = fmaf(qn.x, qn.x, fmaf(qn.y, qn.y, acc));
          } else {
            const float2 y0 = yload(ob + 8 * e);
            const float rx = y0.x - val[e].x, ry = y0.y - val[e].y;
            acc = fmaf(rx, rx, fmaf(ry, ry, acc));
          }
        }
      }
    }
  }
  if (MODE == kFwdLsmr || MODE == kFwdResid)
    wg_sum_store(acc, red, part + (long)series * n_part + blockIdx.x);
}

// H^T (kAdjPlain: xout = H^T y) or one LSMR half-step (kAdjLsmr: p =
// H^T (q u_scale) - v_scale p in place, with norm partials).
template <int MODE>
__global__ __launch_bounds__(kPpfThreads) void ppf_adj_kernel(
    const float2 *__restrict__ yin, float *pio,
    const LsmrState *__restrict__ st, float *__restrict__ part,
    const short *__restrict__ binmap, const float *__restrict__ taps,
    const float2 *__restrict__ tw, int n_sb, long nf, int n_part) {
  __shared__ float2 lds[16 * kPpfFs];
  __shared__ float2 tw_p1[kTwP1], tw_p2[kTwP2];
  __shared__ float red[16];
  // Element offset si nf in y of the subband feeding bin j + 64 q of the
  // packed spectrum (q < 8: bin k = j + 64 q; q >= 8: its mirror 1024 - k),
  // or -1: [q][j].
  __shared__ int soff[16 * 64];

  const int series = blockIdx.y;
  const long F = nf - (kTaps - 1);
  const long N = F * kM;
  const long j0 = (long)blockIdx.x * kPpfWg;
  const long jend = min(j0 + (long)kPpfWg, F);
  const long wend = jend + (kTaps - 1);  // W frames [j0, wend) are used
  const int tid = threadIdx.x;
  const int f = tid & 15, j = tid >> 4;
  const float2 *yi = yin + (long)series * n_sb * nf;
  float *po = pio + (long)series * N;
  fill_tw_tables(tw, tw_p1, tw_p2);  // used after the first pass-0 barrier
  {
    const int q = tid >> 6, b = (tid & 63) + 64 * q;
    const int si = q < 8 ? binmap[b] : (b == 512 ? -1 : binmap[kM - b]);
    soff[tid] = si >= 0 ? si * (int)nf : -1;
  }
  // The series' p through a raw buffer view (32-bit offsets; nf <= 2^19).
  const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(
      po, 0, (int)(N * 4), kRawBufferWord3);
  const char *yb = reinterpret_cast<const char *>(yi);
  __syncthreads();
  // Packing halves, taps g = 1024 h: both folded into the input scale.
  float is = 0.5f / 1024.f, vs = 0.f;
  if (MODE == kAdjLsmr) {
    is *= st[series].u_scale;
    vs = st[series].v_scale;
  }
  float ring[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) ring[i] = 0.f;
  float acc = 0.f;
  const int n_chunk = (int)((wend - j0 + kPpfChunk - 1) / kPpfChunk);
  for (int c = 0; c < n_chunk; ++c) {
    const long mc = j0 + (long)c * kPpfChunk;
    const int jo = opaque(j), fo = opaque(f), ro = opaque(tid);
    const int lo = opaque(tid & 63), wo = opaque(tid >> 6);
    // ---- Packed spectrum of frames mc + 2f, mc + 2f + 1: at bin k,
    // (u_even + i u_odd) / 2; at bin 1024 - k, (conj u_even + i conj
    // u_odd) / 2; zero elsewhere.  Pass 0 reads bins jo + 64 q.
    float2 v[16];
    {
      const int m = (int)mc + 2 * fo;
      const bool in0 = m < (int)nf, in1 = m + 1 < (int)nf;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int o = soff[64 * q + jo];
        float2 a = make_float2(0.f, 0.f), bb = make_float2(0.f, 0.f);
        if (o >= 0) {
          // 32-bit byte offsets from the series base (n_sb nf 8 < 2^31).
          const unsigned ob = (unsigned)(o + m) * 8u;
          if (in0) a = *reinterpret_cast<const float2 *>(yb + ob);
          if (in1) bb = *reinterpret_cast<const float2 *>(yb + ob + 8);
        }
        v[q] = (q < 8) ? make_float2((a.x - bb.y) * is, (a.y + bb.x) * is)
                       : make_float2((a.x + bb.y) * is, (bb.x - a.y) * is);
      }
    }
    dft16<false>(v);
    __syncthreads();  // the previous chunk's reads of lds are done
    {
      float2 *fr = lds + fo * kPpfFs;
#pragma unroll
      for (int q = 0; q < 16; ++q) fr[17 * jo + q] = v[q];  // pad16(16 j + q)
      __syncthreads();
      // Passes 1 and 2: wave w transforms frame w.
      fft1024_wave<false, false>(lds + wo * kPpfFs, tw_p1, tw_p2, lo);
      __syncthreads();
    }
    // ---- Anti-causal FIR: frame jj = m - 15 once W_m has arrived.
    float g[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) g[t] = taps[t * kM + ro];
#pragma unroll
    for (int g8 = 0; g8 < 4; ++g8) {
      float pold[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const long jj = mc + 8 * g8 + i - (kTaps - 1);
        pold[i] = 0.f;
        if (MODE == kAdjLsmr && vs != 0.f && jj >= j0 && jj < jend)
          pold[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
              rp, (unsigned)((int)jj * kM + (kM - 1 - ro)) * 4u, 0, 0));
      }
      float2 w2 = make_float2(0.f, 0.f);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int fi = 8 * g8 + i;
        if (!(fi & 1)) w2 = lds[(fi >> 1) * kPpfFs + pad16(ro)];
        ring[fi & 15] = (fi & 1) ? w2.y : w2.x;
        const long jj = mc + fi - (kTaps - 1);
        if (jj >= j0 && jj < jend) {
          float a = 0.f;
#pragma unroll
          for (int t = 0; t < 16; ++t)
            a = fmaf(g[t], ring[(fi - 15 + t) & 15], a);
          if (MODE == kAdjLsmr) {
            a = fmaf(-vs, pold[i], a);
            acc = fmaf(a, a, acc);
          }
          __builtin_amdgcn_raw_buffer_store_b32(
              __float_as_uint(a), rp,
              (unsigned)((int)jj * kM + (kM - 1 - ro)) * 4u, 0, 0);
        }
      }
    }
  }
  if (MODE == kAdjLsmr)
    wg_sum_store(acc, red, part + (long)series * n_part + blockIdx.x);
}

// Partial sums of |y|^2 (kPpfNormParts contiguous slices per series).
__global__ __launch_bounds__(256) void ppf_sumsq_kernel(
    const float2 *__restrict__ y, long n, float *__restrict__ part) {
  __shared__ float red[4];
  const int series = blockIdx.y;
  const long per = (n + kPpfNormParts - 1) / kPpfNormParts;
  const long a = (long)blockIdx.x * per, b = min(a + per, n);
  const float2 *ys = y + (long)series * n;
  float acc = 0.f;
  for (long i = a + threadIdx.x; i < b; i += 256) {
    const float2 v = ys[i];
    acc = fmaf(v.x, v.x, fmaf(v.y, v.y, acc));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    part[(long)series * kPpfNormParts + blockIdx.x] =
        (red[0] + red[1]) + (red[2] + red[3]);
}

// FP64 sum of n partials by one wave (fixed order; every lane gets it).
__device__ __forceinline__ double wave_sum(const float *part, int n) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += (double)part[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  return s;
}

__device__ __forceinline__ float safe_div(double a, double b) {
  return b != 0.0 ? (float)(a / b) : 0.f;
}

// beta_1 = ||y||; the state starts fresh.
__global__ void lsmr_init_beta_kernel(const float *__restrict__ part,
                                      LsmrState *__restrict__ st) {
  const int series = blockIdx.x;
  const double b2 = wave_sum(part + (long)series * kPpfNormParts,
                             kPpfNormParts);
  if (threadIdx.x != 0) return;
  LsmrState S = {};
  S.beta = sqrt(b2);
  S.u_scale = safe_div(1.0, S.beta);
  S.first = 1;
  S.done = (S.beta == 0.0);
  st[series] = S;
}

// alpha_1 = ||H^T u_1||, and the initial rotation state.
__global__ void lsmr_init_alpha_kernel(const float *__restrict__ part,
                                       int n_part,
                                       LsmrState *__restrict__ st,
                                       double *anorm, int anorm_stride) {
  const int series = blockIdx.x;
  const double a2 = wave_sum(part + (long)series * n_part, n_part);
  if (threadIdx.x != 0) return;
  LsmrState S = st[series];
  S.alpha = S.done ? 0.0 : sqrt(a2);
  if (S.alpha == 0.0) S.done = 1;
  S.alphabar = S.alpha;
  S.zetabar = S.alpha * S.beta;
  S.rho = S.rhobar = S.cbar = 1.0;
  S.sbar = 0.0;
  S.p_scale = safe_div(1.0, S.alpha);
  S.q_scale = safe_div(S.alpha, S.beta);
  S.u_scale = S.v_scale = 0.f;
  S.c_hbar = S.c_x = S.c_h = 0.f;
  S.first = 1;
  st[series] = S;
  if (anorm) anorm[(long)series * anorm_stride] = fabs(S.zetabar);
}

// beta_{k+1} = ||u_{k+1}|| (unnormalised q); scales for the adjoint step.
__global__ void lsmr_beta_kernel(const float *__restrict__ part, int n_part,
                                 LsmrState *__restrict__ st) {
  const int series = blockIdx.x;
  const double b2 = wave_sum(part + (long)series * n_part, n_part);
  if (threadIdx.x != 0) return;
  LsmrState &S = st[series];
  if (S.done) {
    S.u_scale = S.v_scale = 0.f;
    return;
  }
  S.beta = sqrt(b2);
  S.u_scale = safe_div(1.0, S.beta);
  S.v_scale = safe_div(S.beta, S.alpha);
}

// alpha_{k+1} = ||p_{k+1}||, rotations P_k and Pbar_k, and the update
// coefficients of iteration k.
__global__ void lsmr_alpha_kernel(const float *__restrict__ part, int n_part,
                                  LsmrState *__restrict__ st, double *anorm,
                                  int anorm_stride, int k) {
  const int series = blockIdx.x;
  const double a2 = wave_sum(part + (long)series * n_part, n_part);
  if (threadIdx.x != 0) return;
  LsmrState S = st[series];
  double *an = anorm ? anorm + (long)series * anorm_stride : nullptr;
  if (S.done) {
    S.p_scale = S.q_scale = 0.f;
    S.c_hbar = S.c_x = S.c_h = 0.f;
    S.first = 0;
    st[series] = S;
    if (an) an[k] = an[k - 1];
    return;
  }
  const double alpha_new = sqrt(a2);
  // Rotation P_k (no damping: alphahat_k = alphabar_k).
  const double rho_old = S.rho;
  const double rho = hypot(S.alphabar, S.beta);
  const double c = S.alphabar / rho, s = S.beta / rho;
  const double theta_new = s * alpha_new;
  S.alphabar = c * alpha_new;
  // Rotation Pbar_k.
  const double rhobar_old = S.rhobar;
  const double thetabar = S.sbar * rho;
  const double t = S.cbar * rho;
  const double rhobar = hypot(t, theta_new);
  S.cbar = t / rhobar;
  S.sbar = theta_new / rhobar;
  const double zeta = S.cbar * S.zetabar;
  S.zetabar = -S.sbar * S.zetabar;
  // hbar_k = h_k - c_hbar hbar_{k-1}; x_k = x_{k-1} + c_x hbar_k;
  // h_{k+1} = v_{k+1} - c_h h_k.
  S.c_hbar = (float)(thetabar * rho / (rho_old * rhobar_old));
  S.c_x = (float)(zeta / (rho * rhobar));
  S.c_h = (float)(theta_new / rho);
  S.rho = rho;
  S.rhobar = rhobar;
  S.alpha = alpha_new;
  S.p_scale = safe_div(1.0, alpha_new);
  S.q_scale = safe_div(alpha_new, S.beta);
  S.first = 0;
  if (S.beta == 0.0 || alpha_new == 0.0) S.done = 1;
  st[series] = S;
  if (an) an[k] = fabs(S.zetabar);
}

// The last iteration's update of x (x_K = x_{K-1} + c_x (h_K - c_hbar
// hbar_{K-1})); with no iteration done, x = 0.
__global__ __launch_bounds__(256) void lsmr_final_kernel(
    float *__restrict__ x, const float *__restrict__ hv,
    const float *__restrict__ hbar, const LsmrState *__restrict__ st,
    long N) {
  const int series = blockIdx.y;
  const LsmrState &S = st[series];
  const long base = (long)series * N;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  if (S.first) {
    x[base + i] = 0.f;
  } else {
    const float hb = hv[base + i] - S.c_hbar * hbar[base + i];
    x[base + i] = fmaf(S.c_x, hb, x[base + i]);
  }
}

__global__ void ppf_rnorm_kernel(const float *__restrict__ part, int n_part,
                                 double *__restrict__ out) {
  const int series = blockIdx.x;
  const double r2 = wave_sum(part + (long)series * n_part, n_part);
  if (threadIdx.x == 0) out[series] = sqrt(r2);
}

// Station subbands from the staging buffer [n_in][P] (int16 pairs, P =
// n_sb * n_frames positions) to the beamformer's layout [P][n_in] (int8 or
// int16 pairs): 64 positions of every input per workgroup through LDS.
__global__ __launch_bounds__(256) void station_transpose_kernel(
    const short2 *__restrict__ st, long P, int n_in, int ci8,
    void *__restrict__ x) {
  __shared__ short2 tile[64][129];
  const long p0 = (long)blockIdx.x * 64;
  for (int idx = threadIdx.x; idx < 64 * n_in; idx += 256) {
    const int i = idx / 64, pp = idx % 64;
    tile[pp][i] = (p0 + pp < P) ? st[(long)i * P + p0 + pp]
                                : make_short2(0, 0);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * n_in; idx += 256) {
    const int pp = idx / n_in, i = idx % n_in;
    if (p0 + pp >= P) continue;
    const short2 v = tile[pp][i];
    const long o = (p0 + pp) * n_in + i;
    if (ci8) {
      char2 c;
      c.x = (signed char)v.x;
      c.y = (signed char)v.y;
      static_cast<char2 *>(x)[o] = c;
    } else {
      static_cast<short2 *>(x)[o] = v;
    }
  }
}

// The same transpose with 16-byte accesses, for rows of a multiple of 16
// bytes (n_in % 8 == 0 for int8 pairs, n_in % 4 == 0 for int16 pairs) and a
// 16-byte aligned x: each input's 64 positions are read as 16 loads of 4
// positions, and the workgroup's output - 64 consecutive rows, contiguous
// in x - is written as 16-byte chunks (VPC values of one row each).
template <bool CI8>
__global__ __launch_bounds__(256) void station_transpose_vec_kernel(
    const short2 *__restrict__ st, long P, int n_in, void *__restrict__ x) {
  constexpr int VPC = CI8 ? 8 : 4;  // values per 16-byte output chunk
  __shared__ short2 tile[64][129];
  const long p0 = (long)blockIdx.x * 64;
  const bool full = p0 + 64 <= P;
  for (int idx = threadIdx.x; idx < 16 * n_in; idx += 256) {
    const int i = idx >> 4, q = idx & 15;  // positions 4q .. 4q + 3
    const long pp = p0 + 4 * q;
    short2 v[4];
    if (full && ((i * P) & 3) == 0) {
      const int4 w = *reinterpret_cast<const int4 *>(st + (long)i * P + pp);
      v[0] = *reinterpret_cast<const short2 *>(&w.x);
      v[1] = *reinterpret_cast<const short2 *>(&w.y);
      v[2] = *reinterpret_cast<const short2 *>(&w.z);
      v[3] = *reinterpret_cast<const short2 *>(&w.w);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        v[e] = (pp + e < P) ? st[(long)i * P + pp + e] : make_short2(0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) tile[4 * q + e][i] = v[e];
  }
  __syncthreads();
  const int n_chunk = 64 * n_in / VPC;
  char *xb = static_cast<char *>(x) + p0 * n_in * (CI8 ? 2 : 4);
  for (int c = threadIdx.x; c < n_chunk; c += 256) {
    const int e0 = c * VPC, pp = e0 / n_in, i0 = e0 - pp * n_in;
    if (p0 + pp >= P) continue;
    const short2 *t = &tile[pp][i0];
    int4 w;
    if constexpr (CI8) {
      unsigned u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const short2 a = t[2 * k], b = t[2 * k + 1];
        u[k] = (unsigned)(a.x & 0xff) | ((unsigned)(a.y & 0xff) << 8) |
               ((unsigned)(b.x & 0xff) << 16) | ((unsigned)(b.y & 0xff) << 24);
      }
      w = make_int4((int)u[0], (int)u[1], (int)u[2], (int)u[3]);
    } else {
      w = make_int4(*reinterpret_cast<const int *>(&t[0]),
                    *reinterpret_cast<const int *>(&t[1]),
                    *reinterpret_cast<const int *>(&t[2]),
                    *reinterpret_cast<const int *>(&t[3]));
    }
    *reinterpret_cast<int4 *>(xb + (long)c * 16) = w;
  }
}

// ------------------------------------------------------------- host side

struct PpfLayout {
  long F = 0, N = 0;
  int n_fwd = 0, n_adj = 0, n_part = 0;
  size_t st = 0, part = 0, q = 0, p = 0, h = 0, hbar = 0, total = 0;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static PpfLayout ppf_layout(int n_sb, int n_series, long nf) {
  PpfLayout L;
  L.F = nf - (kTaps - 1);
  L.N = L.F * kM;
  L.n_fwd = (int)((nf + kPpfWg - 1) / kPpfWg);
  L.n_adj = (int)((L.F + kPpfWg - 1) / kPpfWg);
  L.n_part = std::max(std::max(L.n_fwd, L.n_adj), kPpfNormParts);
  size_t o = 0;
  L.st = o;
  o = align256(o + (size_t)n_series * kPpfStateBytes);
  L.part = o;
  o = align256(o + (size_t)n_series * L.n_part * 4);
  L.q = o;
  o = align256(o + (size_t)n_series * n_sb * nf * 8);
  L.p = o;
  o = align256(o + (size_t)n_series * L.N * 4);
  L.h = o;
  o = align256(o + (size_t)n_series * L.N * 4);
  L.hbar = o;
  o = align256(o + (size_t)n_series * L.N * 4);
  L.total = o;
  return L;
}

static lp_status ppf_check(const char *who, lp_ctx *ctx, const lp_band *band,
                           int n_series, long nf) {
  if (!ctx) return set_error(LP_EINVAL, "%s: NULL context", who);
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (n_series <= 0 || n_series > 65535)
    return set_error(LP_EINVAL, "%s: n_series %d", who, n_series);
  // The operators address one series with 32-bit byte offsets.
  if (nf < kTaps || nf > kPpfMaxFrames)
    return set_error(LP_EINVAL, "%s: n_frames %ld outside [%d, 2^19]", who,
                     nf, kTaps);
  return LP_OK;
}

static bool aligned(const void *p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

}  // namespace lp

using namespace lp;

extern "C" size_t lp_ppf_work_bytes(int32_t n_sb, int32_t n_series,
                                    int64_t n_frames) {
  if (n_sb <= 0 || n_series <= 0 || n_frames < kTaps) return 0;
  return ppf_layout(n_sb, n_series, n_frames).total;
}

extern "C" lp_status lp_ppf_analyze(lp_ctx *ctx, const lp_band *band,
                                    const float *x, int32_t n_series,
                                    int64_t n_frames, void *y,
                                    void *hip_stream) {
  lp_status rc = ppf_check("lp_ppf_analyze", ctx, band, n_series, n_frames);
  if (rc) return rc;
  if (!x || !y) return set_error(LP_EINVAL, "lp_ppf_analyze: NULL buffer");
  if (!aligned(x, 4) || !aligned(y, 8))
    return set_error(LP_EINVAL, "lp_ppf_analyze: misaligned buffer");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<SynPlan> p;
  if ((rc = get_syn_plan(ctx, band, st, p)) ||
      (rc = plan_wait(p.get(), st)))
    return rc;
  const long nf = n_frames;
  const int n_fwd = (int)((nf + kPpfWg - 1) / kPpfWg);
  hipLaunchKernelGGL(ppf_fwd_kernel<kFwdAnalyze>, dim3(n_fwd, n_series),
                     dim3(kPpfThreads), 0, st, x, (const float2 *)nullptr,
                     static_cast<float2 *>(y), nullptr, nullptr, nullptr,
                     nullptr, nullptr, p->kbin.as<const short>(),
                     p->taps.as<const float>(), ctx->tw4096.as<const float2>(),
                     band->n_sb, nf, 0);
  LP_HIP(hipGetLastError());
  return LP_OK;
}

extern "C" lp_status lp_ppf_adjoint(lp_ctx *ctx, const lp_band *band,
                                    const void *y, int32_t n_series,
                                    int64_t n_frames, float *x,
                                    void *hip_stream) {
  lp_status rc = ppf_check("lp_ppf_adjoint", ctx, band, n_series, n_frames);
  if (rc) return rc;
  if (!x || !y) return set_error(LP_EINVAL, "lp_ppf_adjoint: NULL buffer");
  if (!aligned(x, 4) || !aligned(y, 8))
    return set_error(LP_EINVAL, "lp_ppf_adjoint: misaligned buffer");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<SynPlan> p;
  if ((rc = get_syn_plan(ctx, band, st, p)) ||
      (rc = plan_wait(p.get(), st)))
    return rc;
  const long nf = n_frames, F = nf - (kTaps - 1);
  const int n_adj = (int)((F + kPpfWg - 1) / kPpfWg);
  hipLaunchKernelGGL(ppf_adj_kernel<kAdjPlain>, dim3(n_adj, n_series),
                     dim3(kPpfThreads), 0, st,
                     static_cast<const float2 *>(y), x, nullptr, nullptr,
                     p->binmap.as<const short>(), p->taps.as<const float>(),
                     ctx->tw4096.as<const float2>(), band->n_sb, nf, 0);
  LP_HIP(hipGetLastError());
  return LP_OK;
}

extern "C" lp_status lp_ppf_invert(lp_ctx *ctx, const lp_band *band,
                                   const void *y, int32_t n_series,
                                   int64_t n_frames, int32_t n_iter,
                                   float *x, double *anorm, double *rnorm,
                                   void *work, size_t work_bytes,
                                   void *hip_stream) {
  lp_status rc = ppf_check("lp_ppf_invert", ctx, band, n_series, n_frames);
  if (rc) return rc;
  if (!x || !y || !work)
    return set_error(LP_EINVAL, "lp_ppf_invert: NULL buffer");
  if (n_iter < 0 || n_iter > 100000)
    return set_error(LP_EINVAL, "lp_ppf_invert: n_iter %d", n_iter);
  if (!aligned(x, 4) || !aligned(y, 8) || !aligned(work, 256) ||
      (anorm && !aligned(anorm, 8)) || (rnorm && !aligned(rnorm, 8)))
    return set_error(LP_EINVAL, "lp_ppf_invert: misaligned buffer");
  const long nf = n_frames;
  const int S = band->n_sb;
  const PpfLayout L = ppf_layout(S, n_series, nf);
  if (work_bytes < L.total)
    return set_error(LP_EINVAL, "lp_ppf_invert: work %zu < %zu bytes",
                     work_bytes, L.total);
  if ((rc = set_device(ctx))) return rc;
  hipStream_t hs = static_cast<hipStream_t>(hip_stream);
  PlanRef<SynPlan> p;
  if ((rc = get_syn_plan(ctx, band, hs, p)) ||
      (rc = plan_wait(p.get(), hs)))
    return rc;
  char *w = static_cast<char *>(work);
  LsmrState *st = reinterpret_cast<LsmrState *>(w + L.st);
  float *part = reinterpret_cast<float *>(w + L.part);
  float2 *q = reinterpret_cast<float2 *>(w + L.q);
  float *pv = reinterpret_cast<float *>(w + L.p);
  float *hv = reinterpret_cast<float *>(w + L.h);
  float *hb = reinterpret_cast<float *>(w + L.hbar);
  const float2 *yv = static_cast<const float2 *>(y);
  const short *kbin = p->kbin.as<const short>();
  const short *bmap = p->binmap.as<const short>();
  const float *taps = p->taps.as<const float>();
  const float2 *tw = ctx->tw4096.as<const float2>();
  const int an_stride = n_iter + 1;
  const dim3 gf(L.n_fwd, n_series), ga(L.n_adj, n_series), blk(kPpfThreads);

  // beta_1 u_1 = y; alpha_1 v_1 = H^T u_1.
  hipLaunchKernelGGL(ppf_sumsq_kernel, dim3(kPpfNormParts, n_series),
                     dim3(256), 0, hs, yv, (long)S * nf, part);
  hipLaunchKernelGGL(lsmr_init_beta_kernel, dim3(n_series), dim3(64), 0, hs,
                     part, st);
  hipLaunchKernelGGL(ppf_adj_kernel<kAdjLsmr>, ga, blk, 0, hs, yv, pv, st,
                     part, bmap, taps, tw, S, nf, L.n_adj);
  hipLaunchKernelGGL(lsmr_init_alpha_kernel, dim3(n_series), dim3(64), 0, hs,
                     part, L.n_adj, st, anorm, an_stride);
  for (int k = 1; k <= n_iter; ++k) {
    // beta_{k+1} u_{k+1} = H v_k - alpha_k u_k (u_1 is y itself).
    hipLaunchKernelGGL(ppf_fwd_kernel<kFwdLsmr>, gf, blk, 0, hs, pv,
                       k == 1 ? yv : q, q, hv, hb, x, st, part, kbin, taps,
                       tw, S, nf, L.n_fwd);
    hipLaunchKernelGGL(lsmr_beta_kernel, dim3(n_series), dim3(64), 0, hs,
                       part, L.n_fwd, st);
    // alpha_{k+1} v_{k+1} = H^T u_{k+1} - beta_{k+1} v_k.
    hipLaunchKernelGGL(ppf_adj_kernel<kAdjLsmr>, ga, blk, 0, hs, q, pv, st,
                       part, bmap, taps, tw, S, nf, L.n_adj);
    hipLaunchKernelGGL(lsmr_alpha_kernel, dim3(n_series), dim3(64), 0, hs,
                       part, L.n_adj, st, anorm, an_stride, k);
  }
  hipLaunchKernelGGL(lsmr_final_kernel,
                     dim3((unsigned)((L.N + 255) / 256), n_series), dim3(256),
                     0, hs, x, hv, hb, st, L.N);
  if (rnorm) {
    hipLaunchKernelGGL(ppf_fwd_kernel<kFwdResid>, gf, blk, 0, hs, x, yv,
                       (float2 *)nullptr, nullptr, nullptr, nullptr, st,
                       part, kbin, taps, tw, S, nf, L.n_fwd);
    hipLaunchKernelGGL(ppf_rnorm_kernel, dim3(n_series), dim3(64), 0, hs,
                       part, L.n_fwd, rnorm);
  }
  LP_HIP(hipGetLastError());
  return LP_OK;
}

extern "C" size_t lp_station_work_bytes(int32_t n_in, int32_t n_sb,
                                        int64_t n_frames) {
  if (n_in <= 0 || n_sb <= 0 || n_frames <= 0) return 0;
  return (size_t)n_in * n_sb * n_frames * 4;
}

extern "C" lp_status lp_station_ppf(lp_ctx *ctx, const lp_band *band,
                                    const int16_t *adc, int32_t n_in,
                                    int64_t n_frames, float scale,
                                    int32_t dtype, void *x, void *work,
                                    size_t work_bytes, void *hip_stream) {
  if (!ctx || !adc || !x || !work)
    return set_error(LP_EINVAL, "lp_station_ppf: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (n_in < 1 || n_in > 128)
    return set_error(LP_EINVAL, "lp_station_ppf: n_in %d not in 1..128", n_in);
  if (n_frames < 1 || n_frames > kPpfMaxFrames - 2 * (kTaps - 1))
    return set_error(LP_EINVAL, "lp_station_ppf: n_frames %lld outside "
                     "[1, 2^19 - 30]", (long long)n_frames);
  if (!(scale > 0.f) || !std::isfinite(scale))
    return set_error(LP_EINVAL, "lp_station_ppf: scale must be positive");
  if (dtype != LP_CI8 && dtype != LP_CI16)
    return set_error(LP_EINVAL, "lp_station_ppf: dtype %d", dtype);
  if (work_bytes < lp_station_work_bytes(n_in, band->n_sb, n_frames))
    return set_error(LP_EINVAL, "lp_station_ppf: work %zu bytes too small",
                     work_bytes);
  if (!aligned(adc, 2) || !aligned(x, dtype == LP_CI8 ? 2 : 4) ||
      !aligned(work, 4))
    return set_error(LP_EINVAL, "lp_station_ppf: misaligned buffer");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<SynPlan> p;
  if ((rc = get_syn_plan(ctx, band, st, p)) ||
      (rc = plan_wait(p.get(), st)))
    return rc;
  const long nf = n_frames + 2 * (kTaps - 1);   // frames of H's output
  const int n_fwd = (int)((nf + kPpfWg - 1) / kPpfWg);
  short2 *stage = static_cast<short2 *>(work);
  hipLaunchKernelGGL(ppf_fwd_kernel<kFwdStation>, dim3(n_fwd, n_in),
                     dim3(kPpfThreads), 0, st, adc, (const float2 *)nullptr,
                     (float2 *)nullptr, nullptr, nullptr, nullptr, nullptr,
                     nullptr, p->kbin.as<const short>(),
                     p->taps.as<const float>(), ctx->tw4096.as<const float2>(),
                     band->n_sb, nf, 0, scale, dtype == LP_CI8 ? 128 : 32768,
                     stage);
  const long P = (long)band->n_sb * n_frames;
  const bool ci8 = dtype == LP_CI8;
  const dim3 tgrid((unsigned)((P + 63) / 64));
  if (n_in % (ci8 ? 8 : 4) == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
      reinterpret_cast<uintptr_t>(stage) % 16 == 0) {
    auto *kern = ci8 ? station_transpose_vec_kernel<true>
                     : station_transpose_vec_kernel<false>;
    hipLaunchKernelGGL(kern, tgrid, dim3(256), 0, st, stage, P, (int)n_in, x);
  } else {
    hipLaunchKernelGGL(station_transpose_kernel, tgrid, dim3(256), 0, st, stage,
                       P, (int)n_in, ci8 ? 1 : 0, x);
  }
  LP_HIP(hipGetLastError());
  return LP_OK;
}

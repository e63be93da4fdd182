// Tied-array beamformer (Winchen et al. 2016, Sec. 3, beamforming
// paragraph): per subband k and time t, y_b = sum_i w_{k,i,b} x_{k,t,i}
// with the narrowband weight exp(-2 pi i frac(f_k (r_s . n_b) / c)).
//
// Per subband this is the complex GEMM [n_t x K] . [K x B], run as the real
// GEMM [n_t x 2K] . [2K x 2B]: the input rows are already the interleaved
// (re, im) int samples, and the weight matrix has blocks
// [[w_re, w_im], [-w_im, w_re]].  LP_FP16_MFMA converts the ints to FP16
// (exact for int8) and accumulates in FP32 with v_mfma_f32_16x16x16f16;
// LP_FP32 does the same sums on the vector ALUs.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "lp_internal.h"

namespace lp {

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBfT = 128;        // time rows per tile
constexpr int kBfThreads = 256;  // 4 waves
constexpr size_t kLdsMax = 160 * 1024;

// ------------------------------------------------------------- weights

// st_group / beam_group (both NULL for the regular beamformer): a beam of
// group g weighs only the stations of group g (two-stage beamforming).
__device__ inline void weight_value(const double *__restrict__ enu,
                                    const double *__restrict__ azel,
                                    const float *__restrict__ gain,
                                    const double *__restrict__ wscale,
                                    const int *__restrict__ kk, double f0,
                                    double df, int n_pol, int s, int inp,
                                    int b, const int *__restrict__ st_group,
                                    const int *__restrict__ beam_group,
                                    float &wr, float &wi) {
  int st = inp / n_pol;
  if (st_group && st_group[st] != beam_group[b]) {
    wr = wi = 0.0f;
    return;
  }
  double az = azel[2 * b], el = azel[2 * b + 1];
  double nx = cos(el) * sin(az), ny = cos(el) * cos(az), nz = sin(el);
  double proj = enu[3 * st] * nx + enu[3 * st + 1] * ny + enu[3 * st + 2] * nz;
  double cyc = (f0 + (double)kk[s] * df) * proj / kC;
  float r = (float)(cyc - rint(cyc));  // FP64 range reduction, then FP32
  float sn, cs;
  sincospif(2.0f * r, &sn, &cs);
  float a = (gain ? gain[inp] : 1.0f) * (float)wscale[inp];
  wr = a * cs;
  wi = -a * sn;
}

// MFMA B-operand fragments: element ((s*NT + nt)*KS + ks)*256 + lane*4 + i
// holds Wr[ks*16 + 4*(lane/16) + i][nt*16 + lane%16].
__global__ void bf_weights_mfma_kernel(
    const double *__restrict__ enu, const double *__restrict__ azel,
    const float *__restrict__ gain, const double *__restrict__ wscale,
    const int *__restrict__ kk, double f0, double df, int n_pol, int n_in,
    int n_beams, int n_sb, int KS, int NT, const int *__restrict__ st_group,
    const int *__restrict__ beam_group, _Float16 *__restrict__ wf) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long per_s = (long)NT * KS * 256;
  if (idx >= per_s * n_sb) return;
  int s = (int)(idx / per_s);
  long rem = idx % per_s;
  int nt = (int)(rem / (KS * 256));
  rem %= KS * 256;
  int ks = (int)(rem / 256);
  int lane = (int)(rem % 256) / 4, i = (int)(rem % 4);
  int krow = ks * 16 + 4 * (lane / 16) + i;
  int ncol = nt * 16 + (lane % 16);
  int inp = krow >> 1, xp = krow & 1, b = ncol >> 1, op = ncol & 1;
  float v = 0.0f;
  if (inp < n_in && b < n_beams) {
    float wr, wi;
    weight_value(enu, azel, gain, wscale, kk, f0, df, n_pol, s, inp, b,
                 st_group, beam_group, wr, wi);
    v = (xp == 0) ? (op == 0 ? wr : wi) : (op == 0 ? -wi : wr);
  }
  wf[idx] = (_Float16)v;
}

// FP32 weights [s][in][b] (re, im).
__global__ void bf_weights_fp32_kernel(
    const double *__restrict__ enu, const double *__restrict__ azel,
    const float *__restrict__ gain, const double *__restrict__ wscale,
    const int *__restrict__ kk, double f0, double df, int n_pol, int n_in,
    int n_beams, int n_sb, const int *__restrict__ st_group,
    const int *__restrict__ beam_group, float2 *__restrict__ w) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n_sb * n_in * n_beams) return;
  int b = (int)(idx % n_beams);
  int inp = (int)((idx / n_beams) % n_in);
  int s = (int)(idx / ((long)n_beams * n_in));
  float wr, wi;
  weight_value(enu, azel, gain, wscale, kk, f0, df, n_pol, s, inp, b,
               st_group, beam_group, wr, wi);
  w[idx] = make_float2(wr, wi);
}

// --------------------------------------------------------- MFMA kernel

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// Exact int -> FP16 of one 32-bit word: four int8 (as two half2) or two
// int16 (one half2).  For int8 the biased byte u = x + 128 is placed under
// the FP16 exponent of 1024 (bit pattern 0x6400 | u, value 1024 + u, exact
// since the FP16 ulp at 1024 is 1) and 1152 is subtracted.
template <typename IT>
__device__ __forceinline__ int word_to_half2(unsigned w, half2v *out) {
  if constexpr (sizeof(IT) == 1) {
    unsigned u = w ^ 0x80808080u;
    unsigned lo = __builtin_amdgcn_perm(u, 0x64646464u, 0x00050004u);
    unsigned hi = __builtin_amdgcn_perm(u, 0x64646464u, 0x00070006u);
    half2v a, b;
    __builtin_memcpy(&a, &lo, 4);
    __builtin_memcpy(&b, &hi, 4);
    const half2v off = {(_Float16)1152.0f, (_Float16)1152.0f};
    out[0] = a - off;
    out[1] = b - off;
    return 2;
  } else {
    half2v a;
    a[0] = (_Float16)(short)(w & 0xffffu);
    a[1] = (_Float16)(short)(w >> 16);
    out[0] = a;
    return 1;
  }
}

// Value of lane l ^ 1 (DPP quad_perm 1,0,3,2; a VALU move, no LDS).
__device__ __forceinline__ float lane_swap1(float v) {
  return __int_as_float(
      __builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}

// LDS row stride (bytes) of the staged kernel's raw tile: KS*16 samples
// plus 16 bytes.  For int8 rows the stride in 32-bit words is 4 KS + 4;
// lanes (row r, quarter kq) then read words r (4 KS + 4) + 4 ks + kq.
__host__ __device__ inline int bf_row_stride(int KS, int isz) {
  return KS * 16 * isz + 16;
}

typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx2 __attribute__((ext_vector_type(2)));
template <int VB> struct VecT;
template <> struct VecT<16> { typedef intx4 type; };
template <> struct VecT<8> { typedef intx2 type; };
template <> struct VecT<4> { typedef int type; };

// Grid: x = groups of tiles (T time rows each), y = subband.  Waves are laid
// out WM x WN over (16-row m-tiles, 16-column n-tiles); each wave keeps its
// NPW n-tiles of weight fragments in registers for all of its tiles.  The
// tile's raw integer rows are staged in LDS as loaded (rows of KS*16
// samples, zero padded, plus 16 bytes so row-per-lane fragment reads fall
// on distinct banks) and converted to FP16 as each A fragment is read; the
// next tile is loaded into registers (NV vectors of VB bytes per thread)
// while the current one is multiplied and stored.
template <typename IT, int VB, int NPW, int KSM, int NV>
__global__ __launch_bounds__(kBfThreads) void bf_mfma_kernel(
    const IT *__restrict__ x, const half4 *__restrict__ wf,
    const _Float16 *__restrict__ xscale, int scaled, float2 *__restrict__ y,
    int n_sb, long n_t, long x_nt, int RK, int KS, int NT, int wn_shift,
    int n_beams, int T, int tiles_per_wg, float inv_vpr) {
  typedef typename VecT<VB>::type V;
  constexpr int EPV = VB / (int)sizeof(IT);      // samples per vector
  extern __shared__ __attribute__((aligned(16))) unsigned char smb[];
  const int RSB = bf_row_stride(KSM, (int)sizeof(IT));
  _Float16 *xs_lds = reinterpret_cast<_Float16 *>(smb + T * RSB);
  const int s = blockIdx.y;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  // WN = 2^wn_shift waves across n-tiles, WM = 4 / WN across m-tiles.
  const int WN = 1 << wn_shift;
  const int wn = wave & (WN - 1), wm = wave >> wn_shift;
  const int kq = lane >> 4, col16 = lane & 15;
  const int nvec = T * RK / EPV;
  const int vpr = RK / EPV;  // load vectors per time row

  half4 wreg[NPW][KSM];
#pragma unroll
  for (int p = 0; p < NPW; ++p) {
    int nt = wn + p * WN;
#pragma unroll
    for (int ks = 0; ks < KSM; ++ks) {
      half4 z = {0, 0, 0, 0};
      wreg[p][ks] = (nt < NT && ks < KS)
                        ? wf[((long)(s * NT + nt) * KS + ks) * 64 + lane]
                        : z;
    }
  }
  // Samples RK .. KSM*16-1 of each row multiply zero weights (the weight
  // fragments of k-steps KS .. KSM-1 are zero too); they are zeroed once
  // (the tiles never write them), as are the scale factors past KS*16.
  // Every k-step then runs unconditionally.
  const int padb = (KSM * 16 - RK) * (int)sizeof(IT);
  for (int i = tid; i < T * padb; i += kBfThreads)
    smb[(i / padb) * RSB + RK * (int)sizeof(IT) + (i % padb)] = 0;
  if (scaled)
    for (int i = tid; i < KSM * 16; i += kBfThreads)
      xs_lds[i] = i < KS * 16 ? xscale[i] : (_Float16)0.0f;

  // LDS byte offset of each of this thread's load vectors within a tile
  // (the same for every tile; -1 past the tile).  row = v / vpr through
  // the float reciprocal: exact, since v < 2^12 and the product's error is
  // far below the 0.5 / vpr margin.
  int loff[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int v = tid + kBfThreads * i;
    const int row = (int)(((float)v + 0.5f) * inv_vpr);
    loff[i] = v < nvec ? row * RSB + (v - row * vpr) * VB : -1;
  }
  V pre[NV];
  auto fetch = [&](long t0) {
    // Uniform tile base plus 32-bit per-thread offsets (a tile is at most
    // 16 KB).
    const char *src = reinterpret_cast<const char *>(x) +
                      ((long)s * x_nt + t0) * RK * (long)sizeof(IT);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const unsigned v = tid + kBfThreads * i;
      if (loff[i] >= 0)
        pre[i] = __builtin_nontemporal_load(
            reinterpret_cast<const V *>(src + v * (unsigned)VB));
    }
  };
  auto deposit = [&]() {
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (loff[i] >= 0) *reinterpret_cast<V *>(smb + loff[i]) = pre[i];
  };

  const long tile0 = (long)blockIdx.x * tiles_per_wg;
  if (tile0 * T >= n_t) return;
  fetch(tile0 * T);
  const int mt_per_wave = (T >> 4) >> (2 - wn_shift);
  for (int tile = 0; tile < tiles_per_wg; ++tile) {
    const long t0 = (tile0 + tile) * T;
    if (t0 >= n_t) break;
    __syncthreads();  // the previous tile's LDS reads are done
    deposit();
    // The registers are free once deposited: the next tile's loads go out
    // before the barrier.
    if (tile + 1 < tiles_per_wg && t0 + T < n_t) fetch(t0 + T);
    __syncthreads();
    // The k-steps run without branches (the scaling choice is taken once
    // per tile), so the accumulators stay in place across the MFMA chain.
    auto mtile = [&](int mi, auto sc_c) {
      constexpr bool SC = decltype(sc_c)::value;
      int mt = wm * mt_per_wave + mi;
      int row = mt * 16 + col16;
      const unsigned char *rp = smb + row * RSB;
      floatx4 acc[NPW];
#pragma unroll
      for (int p = 0; p < NPW; ++p) acc[p] = floatx4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KSM; ++ks) {
        // Samples ks*16 + 4*kq .. + 3 of the lane's row.
        half2v h[2];
        if constexpr (sizeof(IT) == 1) {
          word_to_half2<IT>(
              *reinterpret_cast<const unsigned *>(rp + ks * 16 + 4 * kq), h);
        } else {
          uint2 w2 = *reinterpret_cast<const uint2 *>(rp + ks * 32 + 8 * kq);
          word_to_half2<IT>(w2.x, h);
          word_to_half2<IT>(w2.y, h + 1);
        }
        half4 a = {h[0][0], h[0][1], h[1][0], h[1][1]};
        if constexpr (SC)
          a = a * *reinterpret_cast<const half4 *>(xs_lds + ks * 16 + 4 * kq);
#pragma unroll
        for (int p = 0; p < NPW; ++p)
          acc[p] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, wreg[p][ks],
                                                         acc[p], 0, 0, 0);
      }
      // Lane holds D[4 kq + r][col16], r = 0..3.  Even columns are the real
      // parts and odd columns the imaginary parts of beam col/2: each lane
      // takes its neighbour's four values (DPP quad_perm 1,0,3,2: lane l
      // reads lane l ^ 1), so the even lane writes rows 0, 1 and the odd
      // lane rows 2, 3 as two complex each.  (Selecting by component
      // between the lane's own and the neighbour's registers keeps every
      // accumulator index constant.)
#pragma unroll
      for (int p = 0; p < NPW; ++p) {
        int nt = wn + p * WN;
        int col = nt * 16 + col16;
        bool odd = col & 1;
        const float a0 = acc[p][0], a1 = acc[p][1], a2 = acc[p][2],
                    a3 = acc[p][3];
        const float n0 = lane_swap1(a0), n1 = lane_swap1(a1),
                    n2 = lane_swap1(a2), n3 = lane_swap1(a3);
        int b = col >> 1;
        if (nt < NT && b < n_beams) {
          long t = t0 + mt * 16 + 4 * kq + (odd ? 2 : 0);
          const floatx4 o = {odd ? n2 : a0, odd ? a2 : n0, odd ? n3 : a1,
                             odd ? a3 : n1};
          // Streaming store (nontemporal): the beams are read back by the
          // de-dispersion after the whole launch (C2/C4 shapes 7 % faster).
          __builtin_nontemporal_store(
              o, reinterpret_cast<floatx4 *>(y + ((long)b * n_sb + s) * n_t + t));
        }
      }
    };
    if (scaled)
      for (int mi = 0; mi < mt_per_wave; ++mi) mtile(mi, std::true_type());
    else
      for (int mi = 0; mi < mt_per_wave; ++mi) mtile(mi, std::false_type());
  }
}

// --------------------------------------------------------- FP32 kernel

constexpr int kBf32Group = 8;  // beams accumulated per pass over a row

// Grid: x = tiles of T = 256 / G time rows, y = subband.  The tile's raw
// integer samples are staged in LDS with a row stride that is an odd
// number of 32-bit words (conflict-free row-per-lane reads); the weights
// [K][B] follow.  Thread (t, g) forms beams 8g .. 8g + 7, 8(g + G) .. for
// time row t, eight beams per pass over the row.
template <typename IT, int VB>
__global__ __launch_bounds__(kBfThreads) void bf_fp32_kernel(
    const IT *__restrict__ x, const float2 *__restrict__ w,
    float2 *__restrict__ y, int n_sb, long n_t, long x_nt, int n_in,
    int n_beams, int row_words, int G) {
  extern __shared__ int smi[];
  const int T = kBfThreads / G;
  const int RK = 2 * n_in;
  const int row_bytes = RK * (int)sizeof(IT);
  int *xs = smi;                                        // [T][row_words]
  float2 *ws = reinterpret_cast<float2 *>(smi + T * row_words);
  const int s = blockIdx.y;
  const long t0 = (long)blockIdx.x * T;
  const int rows = (int)min((long)T, n_t - t0);
  const char *base =
      reinterpret_cast<const char *>(x + ((long)s * x_nt + t0) * RK);
  const int vec_per_row = row_bytes / VB;
  const int nvec = rows * vec_per_row;
  for (int v = threadIdx.x; v < nvec; v += kBfThreads) {
    int row = v / vec_per_row, c = v - row * vec_per_row;
    int q[VB / 4];
    __builtin_memcpy(q, base + (size_t)v * VB, VB);
#pragma unroll
    for (int i = 0; i < VB / 4; ++i) xs[row * row_words + c * (VB / 4) + i] = q[i];
  }
  const float2 *wsrc = w + (long)s * n_in * n_beams;
  for (int i = threadIdx.x; i < n_in * n_beams; i += kBfThreads) ws[i] = wsrc[i];
  __syncthreads();
  const int t = threadIdx.x % T, g = threadIdx.x / T;
  if (t >= rows) return;
  const int *xr = xs + t * row_words;
  for (int b0 = kBf32Group * g; b0 < n_beams; b0 += kBf32Group * G) {
    float ar[kBf32Group], ai[kBf32Group];
#pragma unroll
    for (int k = 0; k < kBf32Group; ++k) ar[k] = ai[k] = 0.f;
    for (int i = 0; i < n_in; ++i) {
      float re, im;
      if constexpr (sizeof(IT) == 1) {
        int word = xr[i >> 1];
        int sh = (i & 1) * 16;
        re = (float)(signed char)(word >> sh);
        im = (float)(signed char)(word >> (sh + 8));
      } else {
        int word = xr[i];
        re = (float)(short)(word & 0xffff);
        im = (float)(short)(word >> 16);
      }
      const float2 *wi = ws + i * n_beams + b0;
#pragma unroll
      for (int k = 0; k < kBf32Group; ++k) {
        if (b0 + k < n_beams) {
          float2 wv = wi[k];
          ar[k] = fmaf(re, wv.x, ar[k]);
          ar[k] = fmaf(-im, wv.y, ar[k]);
          ai[k] = fmaf(re, wv.y, ai[k]);
          ai[k] = fmaf(im, wv.x, ai[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kBf32Group; ++k)
      if (b0 + k < n_beams)
        y[((long)(b0 + k) * n_sb + s) * n_t + t0 + t] =
            make_float2(ar[k], ai[k]);
  }
}

// ---------------------------------------------------------------- plan

template <typename T>
static void put(std::vector<uint8_t> &v, const T &x) {
  const uint8_t *p = reinterpret_cast<const uint8_t *>(&x);
  v.insert(v.end(), p, p + sizeof(T));
}

lp_status get_bf_plan(lp_ctx *ctx, const lp_array *a, const lp_band *band,
                      const lp_dir *beams, int n_beams, int prec, int dtype,
                      hipStream_t st, PlanRef<BfPlan> &out,
                      const int *st_group, const int *beam_group) {
  const int n_in = a->n_st * a->n_pol;
  const bool fp16_gain = a->gain && prec == LP_FP16_MFMA;
  std::vector<uint8_t> key(1, kPlanBf);
  put(key, prec);
  // The sample type matters only where gains set the FP16 input scaling.
  put(key, fp16_gain ? dtype : 0);
  put(key, (int)(st_group != nullptr));
  if (st_group) {
    for (int i = 0; i < a->n_st; ++i) put(key, st_group[i]);
    for (int b = 0; b < n_beams; ++b) put(key, beam_group[b]);
  }
  put(key, a->n_st);
  put(key, a->n_pol);
  for (int i = 0; i < 3 * a->n_st; ++i) put(key, a->enu_m[i]);
  put(key, (int)(a->gain != nullptr));
  if (a->gain)
    for (int i = 0; i < n_in; ++i) put(key, a->gain[i]);
  put(key, band->n_sb);
  for (int i = 0; i < band->n_sb; ++i) put(key, band->k[i]);
  put(key, band->f0_hz);
  put(key, band->fs_hz);
  put(key, n_beams);
  for (int b = 0; b < n_beams; ++b) {
    put(key, beams[b].az_rad);
    put(key, beams[b].el_rad);
  }

  // Per-input power-of-two scale (FP16 path with gains): e = ceil(log2
  // |a|); the weights are divided by 2^e (|w| <= 1, full FP16 precision,
  // never subnormal) and the samples multiplied by 2^e at conversion
  // (exact).  int8 samples stay within FP16 range for e <= 8 (127 * 2^8).
  // int16 samples would not for any e > 0 (32767 * 2 > 65504), so for them
  // the factor above 1 stays in the weights (|w| <= 2^e <= 256) and only
  // factors below 1 move to the samples.
  std::vector<double> wscale(n_in, 1.0);
  std::vector<_Float16> xscale((size_t)((2 * n_in + 15) / 16) * 16,
                               (_Float16)1.0f);
  bool scaled = false;
  if (fp16_gain) {
    for (int i = 0; i < n_in; ++i) {
      double mag = std::fabs((double)a->gain[i]);
      int e = 0;
      if (mag > 0) e = (int)std::ceil(std::log2(mag));
      if (e < -14 || e > 8)
        return set_error(LP_EINVAL,
                         "gain %g of input %d outside the FP16 scaling range "
                         "(2^-14 .. 2^8 in magnitude, or 0)",
                         (double)a->gain[i], i);
      const int ex = dtype == LP_CI16 ? std::min(e, 0) : e;
      if (ex != 0) scaled = true;
      wscale[i] = std::ldexp(1.0, -ex);
      xscale[2 * i] = xscale[2 * i + 1] = (_Float16)std::ldexp(1.0, ex);
    }
  }

  std::lock_guard<std::mutex> g(ctx->mu);
  out.ctx = ctx;
  if (PlanBase *f = plan_find(ctx, key)) {
    out.p = static_cast<BfPlan *>(f);
    return LP_OK;
  }
  auto p = std::make_unique<BfPlan>();
  p->key = key;
  p->prec = prec;
  p->n_in = n_in;
  p->n_beams = n_beams;
  p->n_sb = band->n_sb;
  p->KS = (2 * n_in + 15) / 16;
  p->NT = (2 * n_beams + 15) / 16;
  p->scaled = scaled;

  // Descriptor copies for the weight kernel, one upload: enu, az/el,
  // weight scale (f64), then subband ids, gains, groups (32-bit).
  std::vector<double> azel(2 * n_beams);
  for (int b = 0; b < n_beams; ++b) {
    azel[2 * b] = beams[b].az_rad;
    azel[2 * b + 1] = beams[b].el_rad;
  }
  size_t o_enu = 0, o_azel = o_enu + 24 * (size_t)a->n_st,
         o_ws = o_azel + 16 * (size_t)n_beams, o_k = o_ws + 8 * (size_t)n_in,
         o_gain = o_k + 4 * (size_t)band->n_sb,
         o_sg = o_gain + (a->gain ? 4 * (size_t)n_in : 0),
         o_bg = o_sg + (st_group ? 4 * (size_t)a->n_st : 0),
         o_end = o_bg + (st_group ? 4 * (size_t)n_beams : 0);
  std::vector<uint8_t> prm(o_end);
  std::memcpy(prm.data() + o_enu, a->enu_m, 24 * (size_t)a->n_st);
  std::memcpy(prm.data() + o_azel, azel.data(), 16 * (size_t)n_beams);
  std::memcpy(prm.data() + o_ws, wscale.data(), 8 * (size_t)n_in);
  std::memcpy(prm.data() + o_k, band->k, 4 * (size_t)band->n_sb);
  if (a->gain) std::memcpy(prm.data() + o_gain, a->gain, 4 * (size_t)n_in);
  if (st_group) {
    std::memcpy(prm.data() + o_sg, st_group, 4 * (size_t)a->n_st);
    std::memcpy(prm.data() + o_bg, beam_group, 4 * (size_t)n_beams);
  }
  lp_status rc;
  if ((rc = plan_alloc(ctx, p.get(), p->params, prm.size())) ||
      (rc = plan_upload(p.get(), p->params, prm.data(), prm.size(), st)))
    return rc;
  const char *P = p->params.as<const char>();
  const double *denu = reinterpret_cast<const double *>(P + o_enu);
  const double *dazel = reinterpret_cast<const double *>(P + o_azel);
  const double *dws = reinterpret_cast<const double *>(P + o_ws);
  const int *dk = reinterpret_cast<const int *>(P + o_k);
  const float *dgain =
      a->gain ? reinterpret_cast<const float *>(P + o_gain) : nullptr;
  const int *dsg = st_group ? reinterpret_cast<const int *>(P + o_sg) : nullptr;
  const int *dbg = st_group ? reinterpret_cast<const int *>(P + o_bg) : nullptr;
  double df = band->fs_hz / kM;
  if (prec == LP_FP16_MFMA) {
    long n = (long)band->n_sb * p->NT * p->KS * 256;
    if ((rc = plan_alloc(ctx, p.get(), p->w, n * 2)) ||
        (rc = plan_alloc(ctx, p.get(), p->xscale, xscale.size() * 2)) ||
        (rc = plan_upload(p.get(), p->xscale, xscale.data(), xscale.size() * 2,
                          st)))
      return rc;
    hipLaunchKernelGGL(bf_weights_mfma_kernel, dim3((n + 255) / 256),
                       dim3(256), 0, st, denu, dazel, dgain, dws, dk,
                       band->f0_hz, df, a->n_pol, n_in, n_beams, band->n_sb,
                       p->KS, p->NT, dsg, dbg, p->w.as<_Float16>());
  } else {
    long n = (long)band->n_sb * n_in * n_beams;
    if ((rc = plan_alloc(ctx, p.get(), p->w, n * 8))) return rc;
    hipLaunchKernelGGL(bf_weights_fp32_kernel, dim3((n + 255) / 256),
                       dim3(256), 0, st, denu, dazel, dgain, dws, dk,
                       band->f0_hz, df, a->n_pol, n_in, n_beams, band->n_sb,
                       dsg, dbg, p->w.as<float2>());
  }
  LP_HIP(hipGetLastError());
  BfPlan *raw = p.get();
  if ((rc = plan_insert(ctx, std::move(p), st))) return rc;
  out.p = raw;
  return LP_OK;
}

template <typename IT>
static lp_status launch_bf(const BfPlan *p, const void *x, long x_nt,
                           long n_t, int n_sb, void *y, hipStream_t st) {
  const int n_in = p->n_in, RK = 2 * n_in;
  const int row_bytes = RK * (int)sizeof(IT);
  const int vb = (row_bytes % 16 == 0) ? 16 : (row_bytes % 8 == 0) ? 8 : 4;
  if (p->prec == LP_FP16_MFMA) {
    const int NT = p->NT, KS = p->KS;
    const int wn_shift = (NT == 1) ? 0 : (NT == 2) ? 1 : 2;
    const int WN = 1 << wn_shift;
    const int npw = (NT + WN - 1) / WN;
    // Rows per tile: at most 64 bytes of input per thread (the prefetch
    // registers), a multiple of 64 rows so the m-tiles split over waves.
    int T = 128;
    while (T > 64 && (long)T * row_bytes > 64L * kBfThreads) T -= 64;
    if ((long)T * row_bytes > 64L * kBfThreads)
      return set_error(LP_EINVAL, "beamformer: %d-byte time rows too long",
                       row_bytes);
    const long tiles = n_t / T;
    // Two tiles per workgroup for a single n-tile (less work per tile,
    // more workgroups in flight), four otherwise: measured on MI355X.
    const int tpw = tiles >= 8 ? (NT == 1 ? 2 : 4) : 1;
    dim3 grid((unsigned)((tiles + tpw - 1) / tpw), n_sb);
    // k-steps per kernel instance (KSM >= KS; the extra ones multiply
    // zeros): the LDS rows hold KSM*16 samples.
    const int ksm = vb == 16 ? (KS <= 6 ? 6 : KS <= 8 ? 8 : KS <= 12 ? 12 : 16)
                             : (KS <= 8 ? 8 : 16);
    size_t shm = (size_t)T * bf_row_stride(ksm, (int)sizeof(IT)) + ksm * 32;
    auto args = [&](auto kern) {
      LP_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shm));
      hipLaunchKernelGGL(kern, grid, dim3(kBfThreads), shm, st,
                         static_cast<const IT *>(x), p->w.as<const half4>(),
                         p->xscale.as<const _Float16>(), (int)p->scaled,
                         static_cast<float2 *>(y), n_sb, n_t, x_nt, RK, KS,
                         NT, wn_shift, p->n_beams, T, tpw,
                         1.0f / (float)(row_bytes / vb));
      return LP_OK;
    };
    // Register arrays sized to the shape: NV load vectors per thread, KSM
    // weight fragments per n-tile.
    const int nv = (int)(((long)T * row_bytes / vb + kBfThreads - 1) /
                         kBfThreads);
    lp_status rc;
    if (vb == 16) {
      auto by_k = [&](auto npw_c, auto nv_c) {
        constexpr int P_ = decltype(npw_c)::value, V_ = decltype(nv_c)::value;
        return KS <= 6    ? args(bf_mfma_kernel<IT, 16, P_, 6, V_>)
               : KS <= 8  ? args(bf_mfma_kernel<IT, 16, P_, 8, V_>)
               : KS <= 12 ? args(bf_mfma_kernel<IT, 16, P_, 12, V_>)
                          : args(bf_mfma_kernel<IT, 16, P_, 16, V_>);
      };
      using C1 = std::integral_constant<int, 1>;
      using C2 = std::integral_constant<int, 2>;
      using C3 = std::integral_constant<int, 3>;
      using C4 = std::integral_constant<int, 4>;
      rc = npw == 1 ? (nv <= 3 ? by_k(C1(), C3()) : by_k(C1(), C4()))
                    : (nv <= 3 ? by_k(C2(), C3()) : by_k(C2(), C4()));
    } else {
      const bool small_k = KS <= 8;
#define LP_BF_PICK(VB_)                                                      \
    (npw == 1 ? (small_k ? args(bf_mfma_kernel<IT, VB_, 1, 8, 64 / VB_>)     \
                         : args(bf_mfma_kernel<IT, VB_, 1, 16, 64 / VB_>))   \
              : (small_k ? args(bf_mfma_kernel<IT, VB_, 2, 8, 64 / VB_>)     \
                         : args(bf_mfma_kernel<IT, VB_, 2, 16, 64 / VB_>)))
      rc = (vb == 8) ? LP_BF_PICK(8) : LP_BF_PICK(4);
#undef LP_BF_PICK
    }
    if (rc) return rc;
  } else {
    int row_words = row_bytes / 4;
    if (row_words % 2 == 0) row_words += 1;  // odd stride: no bank conflicts
    // Rows per tile: 256, halved (with G = 256 / T threads sharing a row's
    // beam groups) until the tile and the weights fit in LDS.
    int T = kBfThreads, G = 1;
    auto lds = [&](int T_) {
      return (size_t)T_ * row_words * 4 + (size_t)n_in * p->n_beams * 8;
    };
    while (lds(T) > kLdsMax && T > 32) {
      T /= 2;
      G *= 2;
    }
    size_t shm = lds(T);
    if (shm > kLdsMax)
      return set_error(LP_EINVAL, "FP32 beamformer tile too large for LDS");
    dim3 grid((unsigned)((n_t + T - 1) / T), n_sb);
    auto args = [&](auto kern) {
      LP_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shm));
      hipLaunchKernelGGL(kern, grid, dim3(kBfThreads), shm, st,
                         static_cast<const IT *>(x), p->w.as<const float2>(),
                         static_cast<float2 *>(y), n_sb, n_t, x_nt, n_in,
                         p->n_beams, row_words, G);
      return LP_OK;
    };
    lp_status rc = (vb == 16)  ? args(bf_fp32_kernel<IT, 16>)
                   : (vb == 8) ? args(bf_fp32_kernel<IT, 8>)
                               : args(bf_fp32_kernel<IT, 4>);
    if (rc) return rc;
  }
  LP_HIP(hipGetLastError());
  return LP_OK;
}

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_beamform(lp_ctx *ctx, const lp_array *array,
                                 const lp_band *band, const lp_dir *beams,
                                 int32_t n_beams, const void *x,
                                 int32_t dtype, int64_t n_t, int32_t prec,
                                 void *y, void *hip_stream) {
  if (!ctx || !array || !beams || !x || !y)
    return set_error(LP_EINVAL, "lp_beamform: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (array->n_st <= 0 || array->n_pol <= 0 || !array->enu_m)
    return set_error(LP_EINVAL, "lp_beamform: bad array descriptor");
  const int n_in = array->n_st * array->n_pol;
  if (n_beams <= 0 || n_beams > 64)
    return set_error(LP_EINVAL, "lp_beamform: n_beams %d not in 1..64",
                     n_beams);
  if (dtype != LP_CI8 && dtype != LP_CI16)
    return set_error(LP_EINVAL, "lp_beamform: dtype %d", dtype);
  if (prec != LP_FP32 && prec != LP_FP16_MFMA)
    return set_error(LP_EINVAL, "lp_beamform: precision %d", prec);
  if (n_t <= 0 || n_t % kBfT != 0)
    return set_error(LP_EINVAL, "lp_beamform: n_t %lld not a multiple of %d",
                     (long long)n_t, kBfT);
  if (const char *why = bf_shape_error(n_in, dtype, prec))
    return set_error(LP_EINVAL, "lp_beamform: %s (n_in %d)", why, n_in);
  if (reinterpret_cast<uintptr_t>(x) % 16 || reinterpret_cast<uintptr_t>(y) % 16)
    return set_error(LP_EINVAL, "lp_beamform: x and y must be 16-byte aligned");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<BfPlan> p;
  if ((rc = get_bf_plan(ctx, array, band, beams, n_beams, prec, dtype, st, p)))
    return rc;
  return bf_launch(p.get(), x, dtype, n_t, 0, n_t, band->n_sb, y, st);
}

namespace lp {
lp_status bf_launch(BfPlan *p, const void *x, int dtype, long x_nt,
                    long x_t0, long n_t, int n_sb, void *y, hipStream_t st) {
  lp_status rc;
  if ((rc = plan_wait(p, st))) return rc;
  if (dtype == LP_CI8)
    return launch_bf<int8_t>(p, static_cast<const int8_t *>(x) +
                                    x_t0 * 2 * p->n_in,
                             x_nt, n_t, n_sb, y, st);
  return launch_bf<int16_t>(p, static_cast<const int16_t *>(x) +
                                   x_t0 * 2 * p->n_in,
                            x_nt, n_t, n_sb, y, st);
}
}  // namespace lp

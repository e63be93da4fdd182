// Station simulator, ADC stage (Winchen et al. 2016, Sec. 2: each station
// samples its antennas at 5 ns; Sec. 5: the simulation chain).  Every input
// (station x polarisation) gets, at absolute sample n,
//   noise = sum_{r < R} (popcount(w_r) - 16)
// with w_r the 32-bit words of Philox4x32-10 (Salmon, Moraes, Dror & Shaw,
// SC 2011) under key (seed lo, seed hi) and counter (n lo, n hi, input,
// group of four words): Binomial(32 R, 1/2) centred, variance 8 R, in
// integer arithmetic, so the codes are reproducible bit for bit anywhere.
// An optional float pulse waveform per input is rounded half to even and
// added; the sum saturates to the ADC's signed range.  The station
// filterbank that turns these codes into subbands is lp_station_ppf.
#include <cmath>

#include "lp_internal.h"

namespace lp {

struct U4 {
  unsigned x, y, z, w;
};

// Philox4x32 with 10 rounds: each round multiplies words 0 and 2 by the two
// round multipliers, mixes the high halves with words 1 and 3 and the key,
// and the key is advanced by the Weyl increments between rounds.
__device__ __forceinline__ U4 philox4x32_10(U4 c, unsigned k0, unsigned k1) {
  const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const unsigned W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    // One 32 x 32 -> 64-bit product gives both halves.
    const unsigned long long p0 = (unsigned long long)M0 * c.x;
    const unsigned long long p1 = (unsigned long long)M1 * c.z;
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__global__ __launch_bounds__(256) void sim_adc_kernel(
    unsigned k0, unsigned k1, int R, int lim, long n0, long n_samp,
    const float *__restrict__ pulse, long pulse_n0, long pulse_len,
    short *__restrict__ adc) {
  const int inp = blockIdx.y;
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_samp) return;
  const unsigned long long n = (unsigned long long)(n0 + t);
  const unsigned lo = (unsigned)n, hi = (unsigned)(n >> 32);
  int acc = 0;
  for (int g = 0; 4 * g < R; ++g) {
    const U4 w = philox4x32_10(U4{lo, hi, (unsigned)inp, (unsigned)g}, k0, k1);
    const unsigned ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * g + j < R) acc += __popc(ws[j]) - 16;
  }
  const long pi = n0 + t - pulse_n0;
  if (pulse && pi >= 0 && pi < pulse_len) {
    // |pulse| is bounded before the conversion (beyond any ADC range).
    const float v = fminf(fmaxf(pulse[(long)inp * pulse_len + pi], -1e6f), 1e6f);
    acc += (int)rintf(v);
  }
  acc = min(max(acc, -lim), lim - 1);
  adc[(long)inp * n_samp + t] = (short)acc;
}

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_sim_adc(lp_ctx *ctx, const lp_sim_cfg *cfg, int64_t n0,
                                int64_t n_samp, const float *pulse,
                                int64_t pulse_n0, int64_t pulse_len,
                                int16_t *adc, void *hip_stream) {
  if (!ctx || !cfg || !adc)
    return set_error(LP_EINVAL, "lp_sim_adc: NULL argument");
  if (cfg->n_in < 1 || cfg->n_in > 65535)
    return set_error(LP_EINVAL, "lp_sim_adc: n_in %d", cfg->n_in);
  if (cfg->noise_words < 0 || cfg->noise_words > 256)
    return set_error(LP_EINVAL, "lp_sim_adc: noise_words %d not in 0..256",
                     cfg->noise_words);
  if (cfg->adc_bits < 2 || cfg->adc_bits > 16)
    return set_error(LP_EINVAL, "lp_sim_adc: adc_bits %d not in 2..16",
                     cfg->adc_bits);
  if (n0 < 0 || n_samp <= 0)
    return set_error(LP_EINVAL, "lp_sim_adc: bad sample range");
  if (pulse && pulse_len <= 0)
    return set_error(LP_EINVAL, "lp_sim_adc: pulse_len must be positive");
  if ((n_samp + 255) / 256 > 0x7fffffffL)
    return set_error(LP_EINVAL, "lp_sim_adc: n_samp too large");
  lp_status rc = set_device(ctx);
  if (rc) return rc;
  const unsigned k0 = (unsigned)(cfg->seed & 0xffffffffu);
  const unsigned k1 = (unsigned)(cfg->seed >> 32);
  dim3 grid((unsigned)((n_samp + 255) / 256), cfg->n_in);
  hipLaunchKernelGGL(sim_adc_kernel, grid, dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), k0, k1,
                     cfg->noise_words, 1 << (cfg->adc_bits - 1), (long)n0,
                     (long)n_samp, pulse, (long)pulse_n0,
                     pulse ? (long)pulse_len : 0L,
                     reinterpret_cast<short *>(adc));
  LP_HIP(hipGetLastError());
  return LP_OK;
}

// De-dispersion and synthesis of one block with memory bounded by one
// beam's group of trials (Winchen et al. 2016, Sec. 3: the STEC search
// repeats the de-dispersion and the inversion for every trial value).
//
// lp_dedisperse holds every trial of every beam at once: B J S n_t complex
// samples, 28.7 GB for 7 beams x 32 trials and 250 GB for 61 x 32.  Here
// the caller's workspace holds G trials of one beam (G S n_t samples): per
// beam and group of trials the de-dispersion fills it and the synthesis
// consumes it into the block's candidate array.  Each group transforms its
// hops forward again, so G trades memory for that repeated work; results
// are those of the two calls made separately up to the rounding of the
// chirp steps (a group's first trial takes its exact chirp).
#include "lp_internal.h"

using namespace lp;

extern "C" size_t lp_ddsyn_work_bytes(int32_t n_sb, int64_t n_t,
                                      int32_t trial_group) {
  if (n_sb <= 0 || n_t <= 0 || trial_group <= 0) return 0;
  return (size_t)trial_group * n_sb * n_t * 8;
}

extern "C" lp_status lp_dedisperse_synthesize(
    lp_ctx *ctx, const lp_band *band, const double *tec_tecu, int32_t n_tec,
    const void *y, int32_t n_beams, int64_t n_t, int64_t frame0, void *tail,
    void *hist, void *cand, int32_t trial_group, void *work,
    size_t work_bytes, void *hip_stream) {
  if (!ctx || !tec_tecu || !y || !tail || !hist || !cand || !work)
    return set_error(LP_EINVAL, "lp_dedisperse_synthesize: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if (n_tec <= 0 || n_tec > 4096)
    return set_error(LP_EINVAL, "lp_dedisperse_synthesize: n_tec %d", n_tec);
  for (int j = 0; j < n_tec; ++j)
    if (!(tec_tecu[j] >= 0.0 && tec_tecu[j] <= 1000.0))
      return set_error(LP_EINVAL,
                       "lp_dedisperse_synthesize: TEC %g outside [0, 1000]",
                       tec_tecu[j]);
  if (n_beams <= 0 || (long)n_beams * n_tec > 65535)
    return set_error(LP_EINVAL,
                     "lp_dedisperse_synthesize: %d beams x %d trials",
                     n_beams, n_tec);
  if (n_t <= 0 || n_t % kHop != 0)
    return set_error(LP_EINVAL,
                     "lp_dedisperse_synthesize: n_t %lld not a positive "
                     "multiple of %d", (long long)n_t, kHop);
  if (frame0 < 0)
    return set_error(LP_EINVAL, "lp_dedisperse_synthesize: frame0 < 0");
  if (trial_group <= 0)
    return set_error(LP_EINVAL, "lp_dedisperse_synthesize: trial_group %d",
                     trial_group);
  const int S = band->n_sb, J = n_tec;
  const int G = trial_group < J ? trial_group : J;
  if (work_bytes < (size_t)G * S * n_t * 8 ||
      reinterpret_cast<uintptr_t>(work) % 16)
    return set_error(LP_EINVAL,
                     "lp_dedisperse_synthesize: work needs %zu bytes, "
                     "16-byte aligned (got %zu)",
                     (size_t)G * S * n_t * 8, work_bytes);
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<DdPlan> dp;
  if ((rc = get_dd_plan(ctx, band, tec_tecu, n_tec, st, dp))) return rc;
  PlanRef<SynPlan> sp;
  if ((rc = get_syn_plan(ctx, band, st, sp))) return rc;
  const float2 *yb = static_cast<const float2 *>(y);
  float2 *tb = static_cast<float2 *>(tail);
  float2 *hb = static_cast<float2 *>(hist);
  for (int b = 0; b < n_beams; ++b) {
    for (int j0 = 0; j0 < J; j0 += G) {
      const int nj = J - j0 < G ? J - j0 : G;
      // Every group reads the previous block's tail; the last one stores
      // this block's.
      const bool last = j0 + nj == J;
      if ((rc = dd_launch(ctx, dp.get(), S, yb + (size_t)b * S * n_t, 1, n_t,
                          tb + (size_t)b * S * kHist, last, work, j0, nj,
                          st)))
        return rc;
      const int q0 = b * J + j0;
      if ((rc = syn_launch(ctx, sp.get(), S, work, nj, n_t, frame0,
                           hb + (size_t)q0 * S * kSynHist, nullptr, cand, n_t,
                           0, q0, n_beams * J, st)))
        return rc;
    }
  }
  return LP_OK;
}

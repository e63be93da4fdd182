// Two-stage beamforming (Winchen et al. 2016, Sec. 4, network paragraph):
// when the link from the station-side cluster cannot carry every station,
// preliminary beams are formed there from subsets of the stations and the
// final beams are formed from them on the processing cluster.
//
// Stage 1 (lp_beamform_groups): for group g and preliminary direction p the
// regular beam over the group's stations only, computed by the beamformer
// kernels with weights that are zero outside the group:
//   y1[g P + p][s][t] = sum_{st in g, pol} w(st, pol, s, n_p) x[s][t][st][pol].
// Stage 2 (lp_beamform_stage2): final beam b takes, from every group, the
// preliminary beam nearest to it (p(b): largest n_p . n_b, lowest p on
// ties) and re-phases it by the group's phase centre r_g (mean station
// position):
//   y[b][s][t] = sum_g exp(-2 pi i frac(f_s r_g . (n_b - n_p(b)) / c))
//                y1[g P + p(b)][s][t].
// The coefficients are formed on the host in FP64 once per plan.  The
// kernel holds one or two time samples of every group's preliminary beam
// in registers and writes every final beam that uses them (coalesced in t).
#include <algorithm>
#include <cmath>

#include "lp_internal.h"

namespace lp {

constexpr int kTsThreads = 256;
constexpr int kTsMaxGroups = 32;

// NS samples per thread (1, or 2 with 16-byte accesses when n_t is even
// and both arrays are 16-byte aligned); GMAX >= G bounds the registers
// that hold the groups' samples.
template <int NS, int GMAX>
__global__ __launch_bounds__(kTsThreads) void ts_stage2_kernel(
    const float2 *__restrict__ y1, const float2 *__restrict__ coef,
    const int *__restrict__ order, const int *__restrict__ pstart, int G,
    int P, int B, int n_sb, long n_t, float2 *__restrict__ y) {
  extern __shared__ float2 cs[];  // [B][G] coefficients of this subband
  const int s = blockIdx.y;
  for (int i = threadIdx.x; i < B * G; i += kTsThreads)
    cs[i] = coef[(long)s * B * G + i];
  __syncthreads();
  const long t = ((long)blockIdx.x * kTsThreads + threadIdx.x) * NS;
  if (t >= n_t) return;
  for (int p = 0; p < P; ++p) {
    const int b0 = pstart[p], b1 = pstart[p + 1];
    if (b0 == b1) continue;
    // v[g][k]: sample t + k of group g's preliminary beam p.
    float2 v[GMAX][NS];
#pragma unroll
    for (int g = 0; g < GMAX; ++g) {
      const float2 *src = y1 + ((long)(g * P + p) * n_sb + s) * n_t + t;
      if constexpr (NS == 2) {
        const float4 q = (g < G) ? *reinterpret_cast<const float4 *>(src)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
        v[g][0] = make_float2(q.x, q.y);
        v[g][1] = make_float2(q.z, q.w);
      } else {
        v[g][0] = (g < G) ? *src : make_float2(0.f, 0.f);
      }
    }
    for (int i = b0; i < b1; ++i) {
      const int b = order[i];
      const float2 *c = cs + b * G;
      float ar[NS], ai[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) ar[k] = ai[k] = 0.f;
#pragma unroll
      for (int g = 0; g < GMAX; ++g) {
        if (g < G) {
          const float2 w = c[g];
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            ar[k] = fmaf(w.x, v[g][k].x, fmaf(-w.y, v[g][k].y, ar[k]));
            ai[k] = fmaf(w.x, v[g][k].y, fmaf(w.y, v[g][k].x, ai[k]));
          }
        }
      }
      float2 *dst = y + ((long)b * n_sb + s) * n_t + t;
      if constexpr (NS == 2)
        *reinterpret_cast<float4 *>(dst) = make_float4(ar[0], ai[0], ar[1], ai[1]);
      else
        *dst = make_float2(ar[0], ai[0]);
    }
  }
}

template <typename T>
static void put(std::vector<uint8_t> &v, const T &x) {
  const uint8_t *p = reinterpret_cast<const uint8_t *>(&x);
  v.insert(v.end(), p, p + sizeof(T));
}

static void unit(const lp_dir &d, double n[3]) {
  n[0] = std::cos(d.el_rad) * std::sin(d.az_rad);
  n[1] = std::cos(d.el_rad) * std::cos(d.az_rad);
  n[2] = std::sin(d.el_rad);
}

static lp_status check_groups(const char *who, const lp_array *a,
                              const lp_groups *gr, int n_prelim) {
  if (!a || !gr || !gr->group || a->n_st <= 0 || a->n_pol <= 0 || !a->enu_m)
    return set_error(LP_EINVAL, "%s: NULL or bad array / groups", who);
  const int G = gr->n_groups;
  if (G < 1 || G > kTsMaxGroups)
    return set_error(LP_EINVAL, "%s: n_groups %d not in 1..%d", who, G,
                     kTsMaxGroups);
  if (n_prelim < 1 || G * n_prelim > 64)
    return set_error(LP_EINVAL,
                     "%s: n_groups * n_prelim = %d * %d not in 1..64", who, G,
                     n_prelim);
  std::vector<int> cnt(G, 0);
  for (int st = 0; st < a->n_st; ++st) {
    int g = gr->group[st];
    if (g < 0 || g >= G)
      return set_error(LP_EINVAL, "%s: station %d in group %d", who, st, g);
    ++cnt[g];
  }
  for (int g = 0; g < G; ++g)
    if (!cnt[g]) return set_error(LP_EINVAL, "%s: group %d is empty", who, g);
  return LP_OK;
}

static lp_status get_ts_plan(lp_ctx *ctx, const lp_array *a,
                             const lp_groups *gr, const lp_band *band,
                             const lp_dir *prelim, int P, const lp_dir *beams,
                             int B, hipStream_t st, PlanRef<TsPlan> &out) {
  const int G = gr->n_groups, S = band->n_sb;
  std::vector<uint8_t> key(1, kPlanTs);
  put(key, a->n_st);
  for (int i = 0; i < 3 * a->n_st; ++i) put(key, a->enu_m[i]);
  put(key, G);
  for (int i = 0; i < a->n_st; ++i) put(key, gr->group[i]);
  put(key, S);
  for (int i = 0; i < S; ++i) put(key, band->k[i]);
  put(key, band->f0_hz);
  put(key, band->fs_hz);
  put(key, P);
  for (int i = 0; i < P; ++i) {
    put(key, prelim[i].az_rad);
    put(key, prelim[i].el_rad);
  }
  put(key, B);
  for (int i = 0; i < B; ++i) {
    put(key, beams[i].az_rad);
    put(key, beams[i].el_rad);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  out.ctx = ctx;
  if (PlanBase *f = plan_find(ctx, key)) {
    out.p = static_cast<TsPlan *>(f);
    return LP_OK;
  }
  auto p = std::make_unique<TsPlan>();
  p->key = key;
  p->G = G;
  p->P = P;
  p->B = B;
  p->S = S;
  // Group phase centres.
  std::vector<double> rg(3 * G, 0.0);
  std::vector<int> cnt(G, 0);
  for (int st = 0; st < a->n_st; ++st) {
    int g = gr->group[st];
    for (int c = 0; c < 3; ++c) rg[3 * g + c] += a->enu_m[3 * st + c];
    ++cnt[g];
  }
  for (int g = 0; g < G; ++g)
    for (int c = 0; c < 3; ++c) rg[3 * g + c] /= cnt[g];
  // Nearest preliminary direction of each final beam.
  std::vector<int> pb(B);
  std::vector<double> np(3 * P);
  for (int i = 0; i < P; ++i) unit(prelim[i], &np[3 * i]);
  for (int b = 0; b < B; ++b) {
    double nb[3];
    unit(beams[b], nb);
    int best = 0;
    double bc = -2.0;
    for (int i = 0; i < P; ++i) {
      double c = nb[0] * np[3 * i] + nb[1] * np[3 * i + 1] + nb[2] * np[3 * i + 2];
      if (c > bc) {
        bc = c;
        best = i;
      }
    }
    pb[b] = best;
  }
  std::vector<int> order(B), pstart(P + 1, 0);
  for (int b = 0; b < B; ++b) ++pstart[pb[b] + 1];
  for (int i = 0; i < P; ++i) pstart[i + 1] += pstart[i];
  {
    std::vector<int> fill(pstart.begin(), pstart.end() - 1);
    for (int b = 0; b < B; ++b) order[fill[pb[b]]++] = b;
  }
  // Coefficients exp(-2 pi i frac(f_s r_g . (n_b - n_p(b)) / c)).
  const double df = band->fs_hz / kM;
  std::vector<float2> coef((size_t)S * B * G);
  for (int s = 0; s < S; ++s) {
    const double f = band->f0_hz + band->k[s] * df;
    for (int b = 0; b < B; ++b) {
      double nb[3];
      unit(beams[b], nb);
      const double *n0 = &np[3 * pb[b]];
      for (int g = 0; g < G; ++g) {
        double proj = rg[3 * g] * (nb[0] - n0[0]) +
                      rg[3 * g + 1] * (nb[1] - n0[1]) +
                      rg[3 * g + 2] * (nb[2] - n0[2]);
        double cyc = f * proj / kC;
        double fr = cyc - std::floor(cyc);
        coef[((size_t)s * B + b) * G + g] =
            make_float2((float)std::cos(2.0 * M_PI * fr),
                        (float)-std::sin(2.0 * M_PI * fr));
      }
    }
  }
  lp_status rc;
  if ((rc = plan_alloc(ctx, p.get(), p->coef, coef.size() * sizeof(float2))) ||
      (rc = plan_upload(p.get(), p->coef, coef.data(),
                        coef.size() * sizeof(float2), st)) ||
      (rc = plan_alloc(ctx, p.get(), p->order, B * 4)) ||
      (rc = plan_upload(p.get(), p->order, order.data(), B * 4, st)) ||
      (rc = plan_alloc(ctx, p.get(), p->pstart, (P + 1) * 4)) ||
      (rc = plan_upload(p.get(), p->pstart, pstart.data(), (P + 1) * 4, st)))
    return rc;
  TsPlan *raw = p.get();
  if ((rc = plan_insert(ctx, std::move(p), st))) return rc;
  out.p = raw;
  return LP_OK;
}

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_beamform_groups(lp_ctx *ctx, const lp_array *array,
                                        const lp_groups *groups,
                                        const lp_band *band,
                                        const lp_dir *prelim,
                                        int32_t n_prelim, const void *x,
                                        int32_t dtype, int64_t n_t,
                                        int32_t prec, void *y1,
                                        void *hip_stream) {
  if (!ctx || !prelim || !x || !y1)
    return set_error(LP_EINVAL, "lp_beamform_groups: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if ((rc = check_groups("lp_beamform_groups", array, groups, n_prelim)))
    return rc;
  const int n_in = array->n_st * array->n_pol;
  if (dtype != LP_CI8 && dtype != LP_CI16)
    return set_error(LP_EINVAL, "lp_beamform_groups: dtype %d", dtype);
  if (prec != LP_FP32 && prec != LP_FP16_MFMA)
    return set_error(LP_EINVAL, "lp_beamform_groups: precision %d", prec);
  if (const char *why = bf_shape_error(n_in, dtype, prec))
    return set_error(LP_EINVAL, "lp_beamform_groups: %s", why);
  if (n_t <= 0 || n_t % 128 != 0)
    return set_error(LP_EINVAL,
                     "lp_beamform_groups: n_t %lld not a multiple of 128",
                     (long long)n_t);
  if (reinterpret_cast<uintptr_t>(x) % 16 ||
      reinterpret_cast<uintptr_t>(y1) % 16)
    return set_error(LP_EINVAL,
                     "lp_beamform_groups: x and y1 must be 16-byte aligned");
  const int G = groups->n_groups, P = n_prelim, NB = G * P;
  std::vector<lp_dir> dirs(NB);
  std::vector<int> bgroup(NB);
  for (int g = 0; g < G; ++g)
    for (int p = 0; p < P; ++p) {
      dirs[g * P + p] = prelim[p];
      bgroup[g * P + p] = g;
    }
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<BfPlan> plan;
  if ((rc = get_bf_plan(ctx, array, band, dirs.data(), NB, prec, dtype, st,
                        plan, groups->group, bgroup.data())))
    return rc;
  return bf_launch(plan.get(), x, dtype, n_t, 0, n_t, band->n_sb, y1, st);
}

extern "C" lp_status lp_beamform_stage2(lp_ctx *ctx, const lp_array *array,
                                        const lp_groups *groups,
                                        const lp_band *band,
                                        const lp_dir *prelim,
                                        int32_t n_prelim,
                                        const lp_dir *beams, int32_t n_beams,
                                        const void *y1, int64_t n_t, void *y,
                                        void *hip_stream) {
  if (!ctx || !prelim || !beams || !y1 || !y)
    return set_error(LP_EINVAL, "lp_beamform_stage2: NULL argument");
  lp_status rc = check_band(band);
  if (rc) return rc;
  if ((rc = check_groups("lp_beamform_stage2", array, groups, n_prelim)))
    return rc;
  if (n_beams < 1 || n_beams > 64)
    return set_error(LP_EINVAL, "lp_beamform_stage2: n_beams %d not in 1..64",
                     n_beams);
  if (n_t <= 0)
    return set_error(LP_EINVAL, "lp_beamform_stage2: n_t %lld",
                     (long long)n_t);
  if (reinterpret_cast<uintptr_t>(y1) % 8 || reinterpret_cast<uintptr_t>(y) % 8)
    return set_error(LP_EINVAL,
                     "lp_beamform_stage2: y1 and y must be 8-byte aligned");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanRef<TsPlan> p;
  if ((rc = get_ts_plan(ctx, array, groups, band, prelim, n_prelim, beams,
                        n_beams, st, p)) ||
      (rc = plan_wait(p.get(), st)))
    return rc;
  const bool two = n_t % 2 == 0 && reinterpret_cast<uintptr_t>(y1) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(y) % 16 == 0;
  const long per_wg = (long)kTsThreads * (two && p->G <= 8 ? 2 : 1);
  dim3 grid((unsigned)((n_t + per_wg - 1) / per_wg), band->n_sb);
  size_t shm = (size_t)p->B * p->G * sizeof(float2);
  // (Two samples of up to 32 groups would take 145 registers.)
  auto *kern = p->G > 8 ? ts_stage2_kernel<1, kTsMaxGroups>
               : two    ? ts_stage2_kernel<2, 8>
                        : ts_stage2_kernel<1, 8>;
  hipLaunchKernelGGL(kern, grid, dim3(kTsThreads), shm, st,
                     static_cast<const float2 *>(y1), p->coef.as<const float2>(),
                     p->order.as<const int>(), p->pstart.as<const int>(),
                     p->G, p->P, p->B, band->n_sb, (long)n_t,
                     static_cast<float2 *>(y));
  LP_HIP(hipGetLastError());
  return LP_OK;
}

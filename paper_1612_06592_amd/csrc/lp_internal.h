// Internal declarations of liblp.so (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lp.h"

namespace lp {

constexpr double kC = 299792458.0;  // speed of light, m/s
constexpr int kM = LP_M;
constexpr int kTaps = LP_TAPS;
constexpr int kNfft = LP_NFFT;
constexpr int kHop = LP_HOP;
constexpr int kDelay = LP_DELAY;
constexpr int kHist = kNfft - kHop;   // overlap-save history per series
constexpr int kSynHist = 16;          // synthesis history frames kept
constexpr int kTrigPerSeries = 256;   // triggers kept per (beam, trial)

// Thread-local error reporting.
lp_status set_error(lp_status code, const char *fmt, ...);
lp_status hip_fail(hipError_t e, const char *what);

#define LP_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return lp::hip_fail(e_, #call); \
  } while (0)

// Device buffer owned by the context.
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
};

// Beam-weight table for one (array, band, beam set, precision).
struct BfPlan {
  std::vector<uint8_t> key;
  int prec = 0;
  int n_in = 0, n_beams = 0, n_sb = 0;
  int KS = 0, NT = 0;        // MFMA: k-steps of 16 real rows, n-tiles of 16
  bool scaled = false;       // per-input power-of-two input scaling in use
  DevBuf w;                  // FP16 MFMA fragments or FP32 [s][in][b]
  DevBuf xscale;             // FP16 [KS*16] input scale factors (MFMA)
};

// Chirp constants for one (band, TEC list).
struct DdPlan {
  std::vector<uint8_t> key;
  int n_tec = 0, n_sb = 0;
  DevBuf base;   // f32 [J][S] frac(kappa T / f_k) in cycles
  DevBuf afac;   // f32 [J][S] kappa T / f_k in cycles
  DevBuf rfk;    // f32 [S] (subband rate / N_fft) / f_k
  DevBuf gq;     // f32 [S][N_fft] x / (1 + x), x = nu_q / f_k (signed bin q)
};

// Synthesis tables for one (band, prototype beta).
struct SynPlan {
  std::vector<uint8_t> key;
  DevBuf taps;    // f32 [16][1024] g = M h
  DevBuf taps2;   // f32 [16][1024] 2 g (synthesis of 2 z)
  DevBuf binmap;  // i16 [512] subband position of bin k, or -1
  DevBuf kbin;    // i16 [n_sb] bin k of each subband position
  int kmax = 511;  // highest bin of the band
};

// Two-stage beamforming: stage-2 coefficients for one (array, grouping,
// band, preliminary and final directions).
struct TsPlan {
  std::vector<uint8_t> key;
  int G = 0, P = 0, B = 0, S = 0;
  DevBuf coef;    // float2 [S][B][G]
  DevBuf order;   // i32 [B] final beams ordered by their preliminary beam
  DevBuf pstart;  // i32 [P + 1] ranges of `order` per preliminary beam
};

}  // namespace lp

struct lp_ctx {
  int device = 0;
  int n_cu = 256;     // compute units of the device
  lp::DevBuf tw4096;  // float2 exp(-2 pi i n / 4096), n < 4096
  std::mutex mu;
  std::vector<std::unique_ptr<lp::BfPlan>> bf;
  std::vector<std::unique_ptr<lp::DdPlan>> dd;
  std::vector<std::unique_ptr<lp::SynPlan>> syn;
  std::vector<std::unique_ptr<lp::TsPlan>> ts;
};

namespace lp {

// Word 3 of a raw (untyped, stride 0) buffer resource on CDNA: 32-bit data
// format, so bounds-checked dword loads are valid (offsets past the
// resource's size read as zero).
constexpr int kRawBufferWord3 = 0x00020000;

// Beamformer input shapes every launch supports: at most 128 inputs, a
// time row (n_in complex samples) a multiple of 4 bytes, and on the
// FP16-MFMA path a row of at most 256 bytes (the kernel's staging tile).
// Returns NULL when supported, else the reason.
inline const char *bf_shape_error(int n_in, int dtype, int prec) {
  if (n_in <= 0 || n_in > 128) return "n_st * n_pol must be in 1..128";
  const int row = 2 * n_in * (dtype == LP_CI8 ? 1 : 2);
  if (row % 4 != 0) return "a time row must be a multiple of 4 bytes";
  if (prec == LP_FP16_MFMA && row > 256)
    return "FP16-MFMA needs time rows of at most 256 bytes "
           "(int16 samples: at most 64 inputs)";
  return nullptr;
}

// Plan lookups (create on first use; creation is synchronous).
lp_status get_bf_plan(lp_ctx *ctx, const lp_array *a, const lp_band *band,
                      const lp_dir *beams, int n_beams, int prec,
                      BfPlan **out, const int *st_group = nullptr,
                      const int *beam_group = nullptr);
lp_status get_dd_plan(lp_ctx *ctx, const lp_band *band, const double *tec,
                      int n_tec, DdPlan **out);
lp_status get_syn_plan(lp_ctx *ctx, const lp_band *band, SynPlan **out);
lp_status check_band(const lp_band *band);
lp_status set_device(lp_ctx *ctx);

// Stage launches on an explicit stream, without argument checks (the
// public entry points and the serving loop validate first).
//   x rows of subband s start at x + (s * x_nt + x_t0) * 2 * n_in samples;
//   cand rows are cand_nt frames long and the block starts at cand_t0.
lp_status bf_launch(const BfPlan *p, const void *x, int dtype, long x_nt,
                    long x_t0, long n_t, int n_sb, void *y, hipStream_t st);
lp_status dd_launch(lp_ctx *ctx, const DdPlan *p, int n_sb, const void *y,
                    int n_beams, long n_t, void *tail, bool update_tail,
                    void *d, hipStream_t st);
lp_status syn_launch(lp_ctx *ctx, const SynPlan *p, int n_sb, const void *d,
                     int n_series, long n_t, long frame0, void *hist,
                     float *x_out, void *cand, long cand_nt, long cand_t0,
                     hipStream_t st);
lp_status trig_launch(const void *cand, int n_beams, int n_tec, long n_t,
                      long frame0, float k_sigma, lp_trig *out, int cap,
                      int *n_out, float *snr_out, int *best_tec,
                      float *sigma_out, void *work, hipStream_t st);

// Remap a linear block index so that consecutive logical blocks land on the
// same XCD (blocks are dealt round-robin over the 8 XCDs of the chip).
__device__ inline long xcd_remap(long bid, long nblocks) {
  const long nx = 8;
  if (nblocks < nx * 2) return bid;
  long per = nblocks / nx;           // full groups per XCD
  long full = per * nx;
  if (bid >= full) return bid;       // leftover tail keeps its index
  return (bid % nx) * per + bid / nx;
}

}  // namespace lp

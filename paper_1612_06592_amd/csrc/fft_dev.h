// Register-level DFT butterflies and Stockham passes shared by the
// de-dispersion (4096-point) and synthesis (1024-point) kernels.
//
// A Stockham pass of radix R over an N-point transform, with Ns the size
// of the sub-transforms already formed, lets butterfly j (0 <= j < N/R)
// read in[j + r N/R], twiddle element r by exp(s 2 pi i (j mod Ns) r /
// (Ns R)), do an R-point DFT and write out[(j / Ns) Ns R + (j mod Ns) +
// r Ns]; Ns = 1, R1, R1 R2, ... yields the natural-order DFT.
#pragma once

#include <hip/hip_runtime.h>

namespace lp {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// 4-point DFT in place; INV selects the +i kernel.
template <bool INV>
__device__ __forceinline__ void dft4(float2 &a, float2 &b, float2 &c,
                                     float2 &d) {
  float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
  a = cadd(t0, t2);
  c = csub(t0, t2);
  if (!INV) {  // X1 = t1 - i t3, X3 = t1 + i t3
    b = make_float2(t1.x + t3.y, t1.y - t3.x);
    d = make_float2(t1.x - t3.y, t1.y + t3.x);
  } else {
    b = make_float2(t1.x - t3.y, t1.y + t3.x);
    d = make_float2(t1.x + t3.y, t1.y - t3.x);
  }
}

// exp(-2 pi i m / 16) for m = 0..15 (cos, -sin).
__device__ __forceinline__ float2 w16(int m) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f,
                  c2 = 0.70710678118654752f;
  switch (m & 15) {
    case 0: return make_float2(1.f, 0.f);
    case 1: return make_float2(c1, -s1);
    case 2: return make_float2(c2, -c2);
    case 3: return make_float2(s1, -c1);
    case 4: return make_float2(0.f, -1.f);
    case 5: return make_float2(-s1, -c1);
    case 6: return make_float2(-c2, -c2);
    case 7: return make_float2(-c1, -s1);
    case 8: return make_float2(-1.f, 0.f);
    case 9: return make_float2(-c1, s1);
    case 10: return make_float2(-c2, c2);
    case 11: return make_float2(-s1, c1);
    case 12: return make_float2(0.f, 1.f);
    case 13: return make_float2(s1, c1);
    case 14: return make_float2(c2, c2);
    default: return make_float2(c1, s1);
  }
}

// v * W16^m (INV: times its conjugate).  W16^4 = -i is a swap and a sign
// change (a general complex product by (0, -1) keeps two products by zero,
// which IEEE arithmetic does not let the compiler drop).
template <bool INV>
__device__ __forceinline__ float2 tw16(float2 v, int m) {
  if (m == 4)
    return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  const float2 w = w16(m);
  return INV ? cmulc(v, w) : cmul(v, w);
}

// First radix-4 stage of a 16-point DFT on inputs x[n2], x[4 + n2],
// x[8 + n2], x[12 + n2] of which only the first K are nonzero (K = 4: the
// full 4-point DFT).  Known zeros are left out of the sums: IEEE arithmetic
// keeps a + 0 (-0 + 0 is +0), so the compiler would not.
template <bool INV, int K>
__device__ __forceinline__ void dft4_first(float2 &a, float2 &b, float2 &c,
                                           float2 &d) {
  if constexpr (K >= 4) {
    dft4<INV>(a, b, c, d);
  } else if constexpr (K == 3) {  // d = 0
    const float2 t0 = cadd(a, c), t1 = csub(a, c);
    a = cadd(t0, b);
    c = csub(t0, b);
    // X1 = t1 -/+ i b, X3 = t1 +/- i b (forward / inverse)
    const float2 ib = make_float2(-b.y, b.x);
    d = INV ? csub(t1, ib) : cadd(t1, ib);
    b = INV ? cadd(t1, ib) : csub(t1, ib);
  } else if constexpr (K == 2) {  // c = d = 0
    const float2 ib = make_float2(-b.y, b.x);
    c = csub(a, b);
    d = INV ? csub(a, ib) : cadd(a, ib);
    const float2 x1 = INV ? cadd(a, ib) : csub(a, ib);
    a = cadd(a, b);
    b = x1;
  } else {  // K == 1: every output is a
    b = a;
    c = a;
    d = a;
  }
}

// 16-point DFT in place, natural order in and out (4 x 4 decomposition:
// n = 4 n1 + n2, k = k1 + 4 k2).  NZ: only inputs 0 .. NZ-1 can be nonzero
// (the others are not read).
template <bool INV, int NZ = 16>
__device__ __forceinline__ void dft16(float2 *v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    // nonzero inputs among n2, n2 + 4, n2 + 8, n2 + 12 (a constant once
    // the loop is unrolled)
    const int k = NZ <= n2 ? 0 : (NZ - n2 + 3) / 4;
    if (k >= 4)
      dft4_first<INV, 4>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    else if (k == 3)
      dft4_first<INV, 3>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    else if (k == 2)
      dft4_first<INV, 2>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    else if (k == 1)
      dft4_first<INV, 1>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    else
      v[n2] = v[4 + n2] = v[8 + n2] = v[12 + n2] = make_float2(0.f, 0.f);
  }
  // v[n2 + 4 k1] now holds A[n2][k1]; apply W16^(n2 k1).
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
      v[n2 + 4 * k1] = tw16<INV>(v[n2 + 4 * k1], n2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
    dft4<INV>(v[4 * k1 + 0], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 index.
  float2 t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[4 * k1 + k2];
}

// Twiddle from the 4096-entry table exp(-2 pi i n / 4096); INV conjugates.
template <bool INV>
__device__ __forceinline__ float2 twiddle(const float2 *__restrict__ tw,
                                          int n) {
  float2 w = tw[n & 4095];
  return INV ? make_float2(w.x, -w.y) : w;
}

// v[r] *= w^r for r = 1..15, with w = table entry `idx` (powers formed by
// repeated multiplication: one load and few live registers; the error
// grows by about one ulp per power).
template <bool INV>
__device__ __forceinline__ void twiddle16(float2 *v,
                                          const float2 *__restrict__ tw,
                                          int idx) {
  const float2 w = twiddle<INV>(tw, idx);
  float2 cur = w;
#pragma unroll
  for (int r = 1; r < 16; ++r) {
    v[r] = cmul(v[r], cur);
    if (r < 15) cur = cmul(cur, w);
  }
}

// Returns x unchanged but hides that from the optimiser, so that loads
// indexed by it are not hoisted out of an enclosing loop (which would keep
// tables of twiddles or taps live in registers across the whole loop).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// LDS index with one pad slot every 16 entries (spreads banks).
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Row swaps across the wavefront (gfx950 v_permlane32/16_swap): with rows
// of 16 lanes, swap_rows32 exchanges rows 2, 3 of a with rows 0, 1 of b;
// swap_rows16 exchanges rows 1, 3 of a with rows 0, 2 of b.
__device__ __forceinline__ void swap_rows32(float2 &a, float2 &b) {
  const auto x = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.x),
                                                  __float_as_uint(b.x), false,
                                                  false);
  const auto y = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.y),
                                                  __float_as_uint(b.y), false,
                                                  false);
  a = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
  b = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
}
__device__ __forceinline__ void swap_rows16(float2 &a, float2 &b) {
  const auto x = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.x),
                                                  __float_as_uint(b.x), false,
                                                  false);
  const auto y = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.y),
                                                  __float_as_uint(b.y), false,
                                                  false);
  a = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
  b = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
}

// After pass 1 of the 1024-point per-wave transform (radix 16, 16, 4), lane
// j holds output (j / 16) 256 + j mod 16 + 16 r in v[r]; the radix-4
// butterfly j + 64 q of pass 2 needs elements j + 64 q + 256 m (m < 4),
// held in v[4 q + j / 16] of lanes j mod 16 + 16 m.  Transposing, in each
// group of four registers, the lane's row of 16 against the register's low
// two bits (two swap steps across rows, no LDS) leaves element
// j + 64 q + 256 m in v[4 q + m].
__device__ __forceinline__ void pass2_gather(float2 *v) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    swap_rows32(v[4 * q], v[4 * q + 2]);
    swap_rows32(v[4 * q + 1], v[4 * q + 3]);
    swap_rows16(v[4 * q], v[4 * q + 1]);
    swap_rows16(v[4 * q + 2], v[4 * q + 3]);
  }
}

}  // namespace lp

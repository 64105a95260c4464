// Device helpers for the Mosaic Flow kernels (gfx950 / CDNA4).
//
// Geometry of the predictor (Sec. 4.1-4.2 of the paper): placements every 16
// cells, 33 x 33 vertices each, four colours, a 128-sample boundary vector
// running counter-clockwise, and the centre-cross / full-interior target
// sets. The tanh used by every kernel is built from the identity
// tanh|x| = (1 - e) / (1 + e), e = exp(-2|x|), with the odd Maclaurin series
// of tanh near zero where that identity cancels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

constexpr int kS = 32;      // cells per unit = cells per subdomain side
constexpr int kHalf = 16;   // placement stride in cells
constexpr int kNB = 128;    // boundary samples per subdomain
constexpr int kCross = 61;  // centre-cross targets
constexpr int kInterior = 961;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// Local (i, j) of boundary sample k (0..127), counter-clockwise from (0, 0).
__device__ __forceinline__ void boundary_local(int k, int& i, int& j) {
  const int side = k >> 5, m = k & 31;
  switch (side) {
    case 0: i = m; j = 0; break;
    case 1: i = kS; j = m; break;
    case 2: i = kS - m; j = kS; break;
    default: i = 0; j = kS - m; break;
  }
}

// Local (i, j) of target t. CROSS: vertical centre line j = 1..31 first, then
// the horizontal line i = 1..31 without the centre. INTERIOR: row by row.
template <int TMODE>
__device__ __forceinline__ void target_local(int t, int& i, int& j) {
  if (TMODE == 0) {
    if (t < 31) { i = kHalf; j = t + 1; }
    else { const int m = t - 31; i = m < 15 ? m + 1 : m + 2; j = kHalf; }
  } else {
    j = t / 31 + 1;
    i = t - (j - 1) * 31 + 1;
  }
}

template <int TMODE>
constexpr int n_targets() { return TMODE == 0 ? kCross : kInterior; }

// Placement q of colour c in a ux x uy domain -> (a, b). Colour (ca, cb)
// holds the placements with a = ca mod 2, b = cb mod 2; there are ux - ca
// of the former and uy - cb of the latter.
__device__ __forceinline__ void placement_of(int q, int colour, int ux, int& a, int& b) {
  const int ca = colour & 1, cb = colour >> 1;
  const int na = ux - ca;
  const int qa = q % na, qb = q / na;
  a = ca + 2 * qa;
  b = cb + 2 * qb;
}

// Number of placements whose interior covers grid index i along one axis of
// n cells: one on stride lines and within half a unit of the ring, else two.
__device__ __forceinline__ float cover_inv(int i, int n) {
  return ((i & 15) == 0 || i < kHalf || i > n - kHalf) ? 1.0f : 0.5f;
}

// float32 tanh: odd series below 0.125, exp-based identity above.
__device__ __forceinline__ float tanh_f32(float x) {
  const float ax = fabsf(x);
  const float x2 = x * x;
  // x - x^3/3 + 2x^5/15 - 17x^7/315 + 62x^9/2835 (Maclaurin series of tanh)
  float p = 62.0f / 2835.0f;
  p = fmaf(p, x2, -17.0f / 315.0f);
  p = fmaf(p, x2, 2.0f / 15.0f);
  p = fmaf(p, x2, -1.0f / 3.0f);
  p = fmaf(p, x2, 0.0f) * x + x;
  // e = 2^(-2 log2(e) |x|) = exp(-2|x|)
  const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * ax);
  const float r = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
  return ax < 0.125f ? p : copysignf(r, x);
}

// GELU(a) = a Phi(a), Phi the standard normal distribution function
// (Phi(a) = (1 + erf(a / sqrt 2)) / 2), with the first two derivatives
// GELU'(a) = Phi(a) + a phi(a) and GELU''(a) = phi(a) (2 - a^2), phi the
// standard normal density. erff is the device library's; the density uses
// the hardware exp2.
__device__ __forceinline__ float gelu_f32(float a) {
  return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f));
}
__device__ __forceinline__ void gelu_rules(float a, float& z, float& d1, float& d2) {
  const float Phi = 0.5f * (1.0f + erff(a * 0.70710678118654752f));
  // phi(a) = e^(-a^2/2) / sqrt(2 pi) = 2^(-a^2 log2(e) / 2) / sqrt(2 pi)
  const float phi = 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * a * a);
  z = a * Phi;
  d1 = fmaf(a, phi, Phi);
  d2 = phi * (2.0f - a * a);
}

// The first three derivatives of GELU: Phi + a phi, phi (2 - a^2) and
// phi a (a^2 - 4) (from phi' = -a phi), for the reverse Taylor rules.
__device__ __forceinline__ void gelu_d123(float a, float& d1, float& d2, float& d3) {
  const float Phi = 0.5f * (1.0f + erff(a * 0.70710678118654752f));
  const float phi = 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * a * a);
  const float a2 = a * a;
  d1 = fmaf(a, phi, Phi);
  d2 = phi * (2.0f - a2);
  d3 = phi * a * (a2 - 4.0f);
}

// Cheaper tanh for activations that are rounded to bf16 next:
// tanh x = 1 - 2 / (1 + exp(2x)); absolute error a few float32 ulps of 1.
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
}

// tanh(x + b) with kb = 2 log2(e) b precomputed: the bias folds into the
// exponent, exp(2 (x + b)) = 2^(2 log2(e) x + kb).
constexpr float kTwoLog2e = 2.8853900817779268f;
__device__ __forceinline__ float tanh_biased(float x, float kb) {
  const float e = __builtin_amdgcn_exp2f(fmaf(x, kTwoLog2e, kb));
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
}

__device__ __forceinline__ floatx16 mfma32x32x2(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx16 mfma32x32x16_bf16(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx16 mfma32x32x16_f16(halfx8 a, halfx8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Row of the 32x32 MFMA accumulator held by lane l in register v.
__device__ __forceinline__ int acc_row(int lane, int v) {
  return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

// float -> bf16, round to nearest even, by the hardware converter
// (v_cvt_pk_bf16_f32 converts two values per instruction).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// float -> fp16, round to nearest even (v_cvt_pk_f16_f32 for pairs).
__device__ __forceinline__ uint16_t f16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (_Float16)f);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bf16_pair(float a, float b, uint16_t& ha, uint16_t& hb) {
  const bf16x2 p = {(__bf16)a, (__bf16)b};
  const uint32_t u = __builtin_bit_cast(uint32_t, p);
  ha = (uint16_t)(u & 0xffffu);
  hb = (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

}  // namespace mf

namespace mf {

// One d x d layer on fp32 MFMA for a tile of 32*RB rows held in LDS (row
// pitch LDH floats). The wave owning output columns [32 w, 32 w + 32)
// passes `wsw` = prepared weights + w * (D/8) * 64 + lane (layout
// [col block][k group][lane][4], see prepare_net_kernel). Inside each
// 8-wide k group lane l feeds k = 8 kg + 4 (l >> 5) + e at MFMA step e to
// both operands, so A and B are read as 16-byte vectors.
template <int D, int RB, int LDH>
__device__ __forceinline__ void mfma_layer_f32(const float* Hs, const floatx4* wsw,
                                               floatx16 (&acc)[RB], int lane) {
  const int arow = lane & 31, ahalf = lane >> 5;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[rb][v] = 0.0f;
#pragma unroll 4
  for (int kg = 0; kg < D / 8; ++kg) {
    const floatx4 bv = wsw[kg * 64];
    floatx4 av[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
      av[rb] = *reinterpret_cast<const floatx4*>(&Hs[(rb * 32 + arow) * LDH + kg * 8 + 4 * ahalf]);
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = mfma32x32x2(av[rb][e], bv[e], acc[rb]);
  }
}

}  // namespace mf

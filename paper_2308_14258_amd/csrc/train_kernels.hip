// Physics-informed SDNet training step on gfx950 (Alg. 1 on one device).
//
// Derivatives with respect to the point (x, y) are propagated forward
// through the network as four streams per point: value v, v_x, v_y and the
// Laplacian v_L. An affine layer maps each stream with the same weights
// (the bias enters the value stream only); tanh maps them by
//   z = tanh a, s = 1 - z^2, z_x = s a_x, z_y = s a_y,
//   z_L = s a_L - 2 z s (a_x^2 + a_y^2),
// so the PDE residual (Eq. 3) is the output layer applied to the Laplacian
// stream. The four streams of a point are stored as four consecutive rows;
// in the 32x32 MFMA accumulator layout those are four consecutive registers
// of one lane, so every tanh rule runs in registers in the GEMM epilogue.
//
// The reverse pass is written out by hand. For the tanh rules above, with
// output adjoints (zb, zb_x, zb_y, zb_L):
//   ab_L = s zb_L
//   ab_x = s (zb_x - 4 z a_x zb_L)
//   ab_y = s (zb_y - 4 z a_y zb_L)
//   ab   = s zb - 2 z s (a_x zb_x + a_y zb_y)
//          - zb_L (2 z s a_L + 2 s (1 - 3 z^2) (a_x^2 + a_y^2))
// and an affine layer gives h-adjoints ab W and weight gradient
// sum_rows ab^T h over all four streams (split-K partial sums, reduced in a
// fixed order: the result is deterministic).
//
// Alg. 1 runs the data points (value stream only) and then the collocation
// points (four streams); both accumulate into one gradient, then Adam.
#include <math.h>

#include <algorithm>

#include "mf_device.h"
#include "mf_internal.h"

namespace mf {


// ---------------------------------------------------------------------------
// W^T of each hidden layer in MFMA operand order (for h-adjoint = ab W).
// ---------------------------------------------------------------------------
__global__ void prepare_wT_kernel(const float* __restrict__ params, int64_t off_w2, int d, float* __restrict__ whT) {
  const int64_t lstride = (int64_t)d * d + d;
  const int64_t dd = (int64_t)d * d;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < 3 * dd;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(idx / dd);
    const int64_t r = idx - l * dd;
    const int e = r & 3, lane = (r >> 2) & 63;
    const int64_t rest = r >> 8;
    const int kg = (int)(rest % (d / 8)), cb = (int)(rest / (d / 8));
    const int j = 32 * cb + (lane & 31);
    const int k = 8 * kg + 4 * (lane >> 5) + e;
    whT[idx] = params[off_w2 + l * lstride + (int64_t)k * d + j];   // (W^T)[j][k] = W[k][j]
  }
}

// ---------------------------------------------------------------------------
// First layer: a = C[b] + x W1x[:,0] + y W1x[:,1]; streams for S = 4 use
// a_x = W1x[:,0], a_y = W1x[:,1], a_L = 0. ACT selects tanh or GELU (for
// GELU: z_x = GELU'(a) a_x, z_L = GELU''(a) (a_x^2 + a_y^2)).
// ---------------------------------------------------------------------------
template <int D, int S, int ACT = ACT_TANH>
__global__ __launch_bounds__(256) void fwd_layer1_kernel(const float* __restrict__ C,
                                                         const float* __restrict__ X, int x_per_bc,
                                                         int64_t rows_per_bc, int64_t n_rows,
                                                         const float* __restrict__ w1x,
                                                         float* __restrict__ Z, float* __restrict__ A1) {
  const int64_t n = n_rows * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / D;
    const int j = (int)(idx - r * D);
    const int64_t b = r / rows_per_bc;
    const float* xp = x_per_bc ? X + 2 * r : X + 2 * (r - b * rows_per_bc);
    const float wx = w1x[2 * j], wy = w1x[2 * j + 1];
    const float a = fmaf(xp[1], wy, fmaf(xp[0], wx, C[b * D + j]));
    if constexpr (ACT == ACT_GELU) {
      float z, d1, d2;
      gelu_rules(a, z, d1, d2);
      if constexpr (S == 1) {
        Z[r * D + j] = z;
        if (A1) A1[r * D + j] = a;
      } else {
        const int64_t o = 4 * r * D + j;
        Z[o] = z;
        if (A1) A1[o] = a;   // the value row of the saved streams (a_x, a_y, a_L are W1x and 0)
        Z[o + D] = d1 * wx;
        Z[o + 2 * D] = d1 * wy;
        Z[o + 3 * D] = d2 * (wx * wx + wy * wy);
      }
      continue;
    }
    const float z = tanh_f32(a);
    if constexpr (S == 1) {
      Z[r * D + j] = z;
    } else {
      const float s = 1.0f - z * z;
      const int64_t o = 4 * r * D + j;
      Z[o] = z;
      Z[o + D] = s * wx;
      Z[o + 2 * D] = s * wy;
      Z[o + 3 * D] = -2.0f * z * s * (wx * wx + wy * wy);
    }
  }
}

// ---------------------------------------------------------------------------
// GEMM over stream rows with a Taylor epilogue.
//   MODE 0 (forward):  P = Zin W^T (+ b on the value stream) -> tanh rules ->
//                      Zout (z streams) and Sv (a_x, a_y, a_L in the rows of
//                      the derivative streams; z is Zout's value row);
//   MODE 1 (backward, value stream only): Zb = Ain W -> Aout = (1 - z^2) Zb.
// The four-stream backward is the fused taylor_bwd_split_kernel /
// taylor_bwd_seq_kernel below.
// A tile is 64 stream rows x D columns, staged in LDS; a persistent grid walks
// the tiles.
// ---------------------------------------------------------------------------
// Register budget for four workgroups per CU (the LDS tile allows four).
template <int D, int S, int MODE, int ACT = ACT_TANH>
__global__ __launch_bounds__(2 * D, 4) void taylor_gemm_kernel(const float* __restrict__ Ain,
                                                            const floatx4* __restrict__ wsw,
                                                            const float* __restrict__ bias,
                                                            const float* __restrict__ Sv_in,
                                                            float* __restrict__ Out,
                                                            float* __restrict__ Sv_out,
                                                            int64_t n_srows, int skip_xy) {
  static_assert(MODE == 0 || S == 1, "four-stream backward: taylor_bwd_*_kernel");
  constexpr int R = 64, RB = 2, LDH = D + 4, NTH = 2 * D;
  constexpr int PER = R * D / 4 / NTH;       // float4 of the input tile per thread
  __shared__ __align__(16) float Hs[R * LDH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n_tiles = (n_srows + R - 1) / R;
  // persistent: tiles blockIdx.x, + gridDim.x, ...; the next tile's input rows
  // are loaded into registers while this tile's MFMAs run
  floatx4 pf[PER];
  auto fetch = [&](int64_t t) {
    const int64_t r0 = t * R;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + i * NTH;
      const int r = idx / (D / 4), c4 = idx - r * (D / 4);
      pf[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
      if (t < n_tiles && r0 + r < n_srows) pf[i] = reinterpret_cast<const floatx4*>(Ain + (r0 + r) * D)[c4];
    }
  };
  fetch(blockIdx.x);
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
  const int64_t row0 = t * R;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = tid + i * NTH;
    const int r = idx / (D / 4), c4 = idx - r * (D / 4);
    *reinterpret_cast<floatx4*>(&Hs[r * LDH + 4 * c4]) = pf[i];
  }
  __syncthreads();
  fetch(t + gridDim.x);

  floatx16 acc[RB];
  mfma_layer_f32<D, RB, LDH>(Hs, wsw + (size_t)wave * (D / 8) * 64 + lane, acc, lane);

  const int j = wave * 32 + (lane & 31);
  const int h = lane >> 5;
  const float bj = (MODE == 0) ? bias[j] : 0.0f;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int64_t sr = row0 + rb * 32 + 8 * m + 4 * h;   // first of 4 consecutive rows
      if constexpr (S == 4) {
        if (sr >= n_srows) continue;
        const int64_t o = sr * D + j;
        if constexpr (MODE == 0 && ACT == ACT_GELU) {
          const float a = acc[rb][4 * m] + bj, ax = acc[rb][4 * m + 1];
          const float ay = acc[rb][4 * m + 2], aL = acc[rb][4 * m + 3];
          float z, d1, d2;
          gelu_rules(a, z, d1, d2);
          Out[o] = z;
          if (!skip_xy) {
            Out[o + D] = d1 * ax;
            Out[o + 2 * D] = d1 * ay;
          }
          Out[o + 3 * D] = fmaf(d2, ax * ax + ay * ay, d1 * aL);
          if (Sv_out) {
            Sv_out[o] = a;   // GELU's rules need the pre-activation, not z
            Sv_out[o + D] = ax;
            Sv_out[o + 2 * D] = ay;
            Sv_out[o + 3 * D] = aL;
          }
        } else if constexpr (MODE == 0) {
          const float a = acc[rb][4 * m] + bj, ax = acc[rb][4 * m + 1];
          const float ay = acc[rb][4 * m + 2], aL = acc[rb][4 * m + 3];
          const float z = tanh_f32(a), s = 1.0f - z * z;
          Out[o] = z;
          if (!skip_xy) {   // the output layer reads only the value and Laplacian streams
            Out[o + D] = s * ax;
            Out[o + 2 * D] = s * ay;
          }
          Out[o + 3 * D] = s * aL - 2.0f * z * s * (ax * ax + ay * ay);
          if (Sv_out) {   // z itself is the value row of Out
            Sv_out[o + D] = ax;
            Sv_out[o + 2 * D] = ay;
            Sv_out[o + 3 * D] = aL;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = sr + e;
          if (row >= n_srows) continue;
          const int64_t o = row * D + j;
          if constexpr (MODE == 0) {
            const float a = acc[rb][4 * m + e] + bj;
            Out[o] = ACT == ACT_GELU ? gelu_f32(a) : tanh_f32(a);
            if (ACT == ACT_GELU && Sv_out) Sv_out[o] = a;
          } else {
            if constexpr (ACT == ACT_GELU) {   // Sv_in: the layer's pre-activations
              float f1, f2, f3;
              gelu_d123(Sv_in[o], f1, f2, f3);
              Out[o] = f1 * acc[rb][4 * m + e];
            } else {                           // Sv_in: the layer's outputs z
              const float z = Sv_in[o];
              Out[o] = (1.0f - z * z) * acc[rb][4 * m + e];
            }
          }
        }
      }
    }
  }
  __syncthreads();   // the next tile overwrites Hs
  }
}

// ---------------------------------------------------------------------------
// Reverse pass of one hidden layer fused with its weight gradient. A
// persistent grid: workgroup b takes the 64-row tiles b, b + gridDim.x, ...
// For each tile the pre-activation adjoints Ab and the layer inputs H are
// staged in LDS once and serve both products:
//   (i)  the input adjoint Ab W (MFMA, weights streamed as in the forward)
//        with the reverse tanh rules of the previous layer -> Out;
//   (ii) the weight gradient P[j][k] += sum_r Ab[r][j] H[r][k], held in
//        MFMA accumulators across the workgroup's tiles (wave w owns rows
//        j in [32 w, 32 w + 32) and all column blocks), and the bias
//        gradient sum over value rows of Ab.
// Each workgroup writes one partial; the partials are summed in workgroup
// order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------

// Reverse tanh rules of the previous layer applied to Zb = Ab W (acc). z is
// that layer's output, i.e. the value rows of the layer-input tile `HH`
// (LDS, row pitch LDH); a_x, a_y, a_L come from the saved streams Sv_in, or,
// when Sv_in is null (the previous layer is the first one, whose stream
// derivatives do not depend on the row), a_x = W1x[j][0], a_y = W1x[j][1],
// a_L = 0 (L1: the previous layer is the first one).
template <int D, int S, int LDH, bool L1, int ACT = ACT_TANH>
__device__ __forceinline__ void bwd_epilogue(const floatx16 (&acc)[2], int64_t row0, int j, int h,
                                             const float* HH, const float* __restrict__ Sv_in,
                                             const float* __restrict__ w1x, float* __restrict__ Out,
                                             int64_t n_srows) {
  float ax1 = 0.0f, ay1 = 0.0f;
  if constexpr (S == 4 && L1) {
    ax1 = w1x[2 * j];
    ay1 = w1x[2 * j + 1];
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int lr = rb * 32 + 8 * m + 4 * h;                // first of 4 consecutive rows in the tile
      const int64_t sr = row0 + lr;
      if constexpr (S == 4) {
        if (sr >= n_srows) continue;
        const int64_t o = sr * D + j;
        const float ax = L1 ? ax1 : Sv_in[o + D], ay = L1 ? ay1 : Sv_in[o + 2 * D];
        const float aL = L1 ? 0.0f : Sv_in[o + 3 * D];
        const float zb = acc[rb][4 * m], zbx = acc[rb][4 * m + 1];
        const float zby = acc[rb][4 * m + 2], zbL = acc[rb][4 * m + 3];
        if constexpr (ACT == ACT_GELU) {
          // f1, f2, f3: GELU's first three derivatives at the saved pre-activation
          float f1, f2, f3;
          gelu_d123(Sv_in[o], f1, f2, f3);
          const float q = ax * ax + ay * ay;
          Out[o] = f1 * zb + f2 * (ax * zbx + ay * zby) + zbL * (f2 * aL + f3 * q);
          Out[o + D] = f1 * zbx + 2.0f * f2 * ax * zbL;
          Out[o + 2 * D] = f1 * zby + 2.0f * f2 * ay * zbL;
          Out[o + 3 * D] = f1 * zbL;
          continue;
        }
        const float z = HH[lr * LDH + j];
        const float s = 1.0f - z * z, q = ax * ax + ay * ay;
        Out[o] = s * zb - 2.0f * z * s * (ax * zbx + ay * zby) -
                 zbL * (2.0f * z * s * aL + 2.0f * s * (1.0f - 3.0f * z * z) * q);
        Out[o + D] = s * (zbx - 4.0f * z * ax * zbL);
        Out[o + 2 * D] = s * (zby - 4.0f * z * ay * zbL);
        Out[o + 3 * D] = s * zbL;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = sr + e;
          if (row >= n_srows) continue;
          if constexpr (ACT == ACT_GELU) {
            float f1, f2, f3;
            gelu_d123(Sv_in[row * D + j], f1, f2, f3);
            Out[row * D + j] = f1 * acc[rb][4 * m + e];
          } else {
            const float z = HH[(lr + e) * LDH + j];
            Out[row * D + j] = (1.0f - z * z) * acc[rb][4 * m + e];
          }
        }
      }
    }
  }
}

// Register budget for two 8-wave workgroups per CU (four waves per SIMD).
template <int D, int S, bool L1, int ACT = ACT_TANH>
__global__ __launch_bounds__(4 * D, 4) void taylor_bwd_split_kernel(const float* __restrict__ Ab,
                                                           const float* __restrict__ H,
                                                           const floatx4* __restrict__ wsw,
                                                           const float* __restrict__ Sv_in,
                                                           const float* __restrict__ w1x,
                                                           float* __restrict__ Out, int64_t n_srows,
                                                           float* __restrict__ wpart,
                                                           float* __restrict__ bpart) {
  // Two roles of D/32 waves each, running concurrently on the same staged
  // tile: waves [0, D/32) form the input adjoint (and load the Ab rows),
  // waves [D/32, 2 D/32) the weight gradient (and load the H rows). Each
  // role runs its own loop with the same barriers, so each keeps only its
  // own accumulators in registers.
  constexpr int R = 64, RB = 2, LDH = D + 4, NW = D / 32, NKB = D / 32;
  constexpr int RTH = 64 * NW;                 // threads per role
  constexpr int PER = R * D / 4 / RTH;         // float4 per thread of one tile array
  __shared__ __align__(16) float HA[R * LDH];
  __shared__ __align__(16) float HH[R * LDH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, h = lane >> 5;
  const int64_t n_tiles = (n_srows + R - 1) / R;
  // The adjoint role stages its tile array (Ab) from registers filled one
  // tile ahead: the loads of tile t + gridDim.x are issued before tile t's
  // MFMAs. The weight-gradient role, which holds D/32 accumulator blocks,
  // loads its array (H) at the top of each tile.
  floatx4 pf[PER];
  auto fetch = [&](const float* src, int rt, int64_t t) {
    const int64_t row0 = t * R;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = rt + i * RTH;
      const int r = idx / (D / 4), c4 = idx - r * (D / 4);
      pf[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
      if (t < n_tiles && row0 + r < n_srows) pf[i] = reinterpret_cast<const floatx4*>(src + (row0 + r) * D)[c4];
    }
  };
  auto stage = [&](float* dst, int rt) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = rt + i * RTH;
      const int r = idx / (D / 4), c4 = idx - r * (D / 4);
      *reinterpret_cast<floatx4*>(&dst[r * LDH + 4 * c4]) = pf[i];
    }
  };
  if (wave < NW) {
    const int rt = tid;                        // thread within the role
    const int j = wave * 32 + col;
    fetch(Ab, rt, blockIdx.x);
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
      const int64_t row0 = t * R;
      stage(HA, rt);
      __syncthreads();
      fetch(Ab, rt, t + gridDim.x);
      floatx16 acc[RB];
      mfma_layer_f32<D, RB, LDH>(HA, wsw + (size_t)wave * (D / 8) * 64 + lane, acc, lane);
      bwd_epilogue<D, S, LDH, L1, ACT>(acc, row0, j, h, HH, Sv_in, w1x, Out, n_srows);
      __syncthreads();   // the next tile overwrites the LDS
    }
  } else {
    const int rt = tid - RTH;
    const int jw = wave - NW;                  // output rows j in [32 jw, 32 jw + 32)
    const int j = jw * 32 + col;
    floatx16 accw[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int v = 0; v < 16; ++v) accw[kb][v] = 0.0f;
    float bsum = 0.0f;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
      fetch(H, rt, t);
      stage(HH, rt);
      __syncthreads();
      // weight gradient over the tile's rows: lane feeds row 8 g + 4 h + e
      // at MFMA step e to both operands
#pragma unroll 2
      for (int g = 0; g < R / 8; ++g) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 8 * g + 4 * h + e;
          const float a = HA[r * LDH + j];
#pragma unroll
          for (int kb = 0; kb < NKB; ++kb) accw[kb] = mfma32x32x2(a, HH[r * LDH + kb * 32 + col], accw[kb]);
        }
      }
      if (rt < D)
        for (int r = 0; r < R; r += S) bsum += HA[r * LDH + rt];   // value rows (zero beyond the end)
      __syncthreads();
    }
    float* P = wpart + (int64_t)blockIdx.x * D * D;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int v = 0; v < 16; ++v) P[(int64_t)(jw * 32 + acc_row(lane, v)) * D + kb * 32 + col] = accw[kb][v];
    if (rt < D) bpart[(int64_t)blockIdx.x * D + rt] = bsum;
  }
}

// Width 256: one role per wave (both products in turn); the role-split
// form above would need more than the 128 VGPRs a 1024-thread workgroup
// allows.
template <int D, int S, bool L1, int ACT = ACT_TANH>
__global__ __launch_bounds__(2 * D) void taylor_bwd_seq_kernel(const float* __restrict__ Ab,
                                                           const float* __restrict__ H,
                                                           const floatx4* __restrict__ wsw,
                                                           const float* __restrict__ Sv_in,
                                                           const float* __restrict__ w1x,
                                                           float* __restrict__ Out, int64_t n_srows,
                                                           float* __restrict__ wpart,
                                                           float* __restrict__ bpart) {
  constexpr int R = 64, RB = 2, LDH = D + 4, NTH = 2 * D, NKB = D / 32;
  __shared__ __align__(16) float HA[R * LDH];
  __shared__ __align__(16) float HH[R * LDH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, h = lane >> 5;
  const int j = wave * 32 + col;
  floatx16 accw[NKB];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int v = 0; v < 16; ++v) accw[kb][v] = 0.0f;
  float bsum = 0.0f;
  const int64_t n_tiles = (n_srows + R - 1) / R;
  // the next tile's adjoint rows are loaded into registers while this one
  // computes (the input rows follow with the LDS stores)
  constexpr int PER = R * D / 4 / NTH;   // float4 per thread per array
  floatx4 pa[PER];
  auto fetch = [&](int64_t t) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + i * NTH;
      const int r = idx / (D / 4), c4 = idx - r * (D / 4);
      const int64_t row = t * R + r;
      pa[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
      if (t < n_tiles && row < n_srows) pa[i] = reinterpret_cast<const floatx4*>(Ab + row * D)[c4];
    }
  };
  fetch(blockIdx.x);
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t row0 = t * R;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + i * NTH;
      const int r = idx / (D / 4), c4 = idx - r * (D / 4);
      floatx4 vh = {0.0f, 0.0f, 0.0f, 0.0f};
      if (row0 + r < n_srows) vh = reinterpret_cast<const floatx4*>(H + (row0 + r) * D)[c4];
      *reinterpret_cast<floatx4*>(&HA[r * LDH + 4 * c4]) = pa[i];
      *reinterpret_cast<floatx4*>(&HH[r * LDH + 4 * c4]) = vh;
    }
    __syncthreads();
    fetch(t + gridDim.x);
    // (i) input adjoint and reverse rules
    floatx16 acc[RB];
    mfma_layer_f32<D, RB, LDH>(HA, wsw + (size_t)wave * (D / 8) * 64 + lane, acc, lane);
    bwd_epilogue<D, S, LDH, L1, ACT>(acc, row0, j, h, HH, Sv_in, w1x, Out, n_srows);
    // (ii) weight gradient over the tile's rows: lane feeds row 8 g + 4 h + e
    // at MFMA step e to both operands
#pragma unroll 2
    for (int g = 0; g < R / 8; ++g) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 8 * g + 4 * h + e;
        const float a = HA[r * LDH + j];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) accw[kb] = mfma32x32x2(a, HH[r * LDH + kb * 32 + col], accw[kb]);
      }
    }
    if (tid < D)
      for (int r = 0; r < R; r += S) bsum += HA[r * LDH + tid];   // value rows (zero beyond the end)
    __syncthreads();   // the next tile overwrites the LDS
  }
  float* P = wpart + (int64_t)blockIdx.x * D * D;
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int v = 0; v < 16; ++v) P[(int64_t)(wave * 32 + acc_row(lane, v)) * D + kb * 32 + col] = accw[kb][v];
  if (tid < D) bpart[(int64_t)blockIdx.x * D + tid] = bsum;
}

// ---------------------------------------------------------------------------
// Output layer, loss and the seed of the reverse pass. One wave per point.
//   S = 4 (collocation): residual u_L = w5 . z_L; ub_L = 2 u_L / n.
//   S = 1 (data):        residual u - g; ub = 2 (u - g) / n.
// Writes ab_4 = reverse tanh rules of zb_4 = w5 ub, and per-wave partial
// sums of the w5 / b5 gradient and of the squared residual.
// ---------------------------------------------------------------------------
template <int D, int S, int ACT = ACT_TANH>
__global__ __launch_bounds__(256) void output_loss_kernel(const float* __restrict__ Z4,
                                                          const float* __restrict__ Sv4,
                                                          const float* __restrict__ w5,
                                                          const float* __restrict__ b5,
                                                          const float* __restrict__ target,
                                                          int64_t n_rows, float inv_n,
                                                          float* __restrict__ Ab,
                                                          float* __restrict__ opart) {
  constexpr int NJ = D / 64;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  float w5r[NJ], gw5[NJ];
#pragma unroll
  for (int t = 0; t < NJ; ++t) {
    w5r[t] = w5[lane + 64 * t];
    gw5[t] = 0.0f;
  }
  float gb5 = 0.0f, lsum = 0.0f;
  for (int64_t r = gw; r < n_rows; r += kOutWaves) {
    if constexpr (S == 4) {
      const int64_t o = 4 * r * D;
      float zL[NJ], p = 0.0f;
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        zL[t] = Z4[o + 3 * D + lane + 64 * t];
        p = fmaf(w5r[t], zL[t], p);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off);
      const float res = p;                      // Laplacian of the output
      lsum = fmaf(res, res, lsum);
      const float ubL = 2.0f * res * inv_n;
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        const int j = lane + 64 * t;
        gw5[t] = fmaf(ubL, zL[t], gw5[t]);
        const float ax = Sv4[o + D + j], ay = Sv4[o + 2 * D + j];
        const float aL = Sv4[o + 3 * D + j];
        const float zbL = w5r[t] * ubL;
        if constexpr (ACT == ACT_GELU) {   // only z_L carries an adjoint here
          float f1, f2, f3;
          gelu_d123(Sv4[o + j], f1, f2, f3);
          Ab[o + j] = zbL * (f2 * aL + f3 * (ax * ax + ay * ay));
          Ab[o + D + j] = 2.0f * f2 * ax * zbL;
          Ab[o + 2 * D + j] = 2.0f * f2 * ay * zbL;
          Ab[o + 3 * D + j] = f1 * zbL;
          continue;
        }
        const float z = Z4[o + j];
        const float s = 1.0f - z * z, q = ax * ax + ay * ay;
        Ab[o + j] = -zbL * (2.0f * z * s * aL + 2.0f * s * (1.0f - 3.0f * z * z) * q);
        Ab[o + D + j] = s * (-4.0f * z * ax * zbL);
        Ab[o + 2 * D + j] = s * (-4.0f * z * ay * zbL);
        Ab[o + 3 * D + j] = s * zbL;
      }
    } else {
      const int64_t o = r * D;
      float zv[NJ], p = 0.0f;
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        zv[t] = Z4[o + lane + 64 * t];
        p = fmaf(w5r[t], zv[t], p);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off);
      const float res = p + b5[0] - target[r];
      lsum = fmaf(res, res, lsum);
      const float ub = 2.0f * res * inv_n;
      gb5 += ub;
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        gw5[t] = fmaf(ub, zv[t], gw5[t]);
        if constexpr (ACT == ACT_GELU) {
          float f1, f2, f3;
          gelu_d123(Sv4[o + lane + 64 * t], f1, f2, f3);
          Ab[o + lane + 64 * t] = f1 * w5r[t] * ub;
        } else {
          Ab[o + lane + 64 * t] = (1.0f - zv[t] * zv[t]) * w5r[t] * ub;
        }
      }
    }
  }
  float* op = opart + (int64_t)gw * (D + 2);
#pragma unroll
  for (int t = 0; t < NJ; ++t) op[lane + 64 * t] = gw5[t];
  if (lane == 0) {
    op[D] = gb5;
    op[D + 1] = lsum;
  }
}

// out[i] (+)= sum_p part[p * stride + i]. Eight threads per element each sum
// the partials p = g, g + 8, ... and the eight sums are added in g order, so
// the result does not depend on the launch shape.
constexpr int kReduceGroups = 8;

__global__ __launch_bounds__(256) void reduce_parts_kernel(const float* __restrict__ part, int64_t n_parts,
                                                           int64_t n, int64_t stride, float* __restrict__ out,
                                                           int accumulate) {
  constexpr int EPB = 256 / kReduceGroups;   // elements per block
  __shared__ float sh[kReduceGroups][EPB];
  const int e = threadIdx.x % EPB, g = threadIdx.x / EPB;
  for (int64_t i0 = (int64_t)blockIdx.x * EPB; i0 < n; i0 += (int64_t)gridDim.x * EPB) {
    const int64_t i = i0 + e;
    float s = 0.0f;
    if (i < n) {
#pragma unroll 8
      for (int64_t p = g; p < n_parts; p += kReduceGroups) s += part[p * stride + i];
    }
    sh[g][e] = s;
    __syncthreads();
    if (g == 0 && i < n) {
      float t = 0.0f;
#pragma unroll
      for (int q = 0; q < kReduceGroups; ++q) t += sh[q][e];
      out[i] = accumulate ? out[i] + t : t;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// First-layer reductions per boundary condition b:
//   c[b][j]  = sum_rows ab,  cx[b][j] = sum_rows (ab x + ab_x),
//   cy[b][j] = sum_rows (ab y + ab_y).
// One workgroup per condition: kL1Groups row groups of D threads each sum a
// contiguous quarter of the condition's rows, then the group sums are added
// in group order.
// ---------------------------------------------------------------------------
constexpr int kL1Groups = 4;

template <int D, int S>
__global__ __launch_bounds__(kL1Groups * D) void layer1_reduce_kernel(const float* __restrict__ Ab1,
                                                                     const float* __restrict__ X, int x_per_bc,
                                                                     int64_t rows_per_bc, int64_t B,
                                                                     float* __restrict__ out) {
  __shared__ float red[3][kL1Groups][D];
  const int64_t b = blockIdx.x;
  const int j = threadIdx.x % D, grp = threadIdx.x / D;
  const int64_t per = (rows_per_bc + kL1Groups - 1) / kL1Groups;
  const int64_t p0 = grp * per, p1 = std::min<int64_t>(rows_per_bc, p0 + per);
  float c = 0.0f, cx = 0.0f, cy = 0.0f;
#pragma unroll 4
  for (int64_t p = p0; p < p1; ++p) {
    const int64_t r = b * rows_per_bc + p;
    const float* xp = x_per_bc ? X + 2 * r : X + 2 * p;
    const float a = Ab1[S * r * D + j];
    float ax = 0.0f, ay = 0.0f;
    if constexpr (S == 4) {
      ax = Ab1[(4 * r + 1) * D + j];
      ay = Ab1[(4 * r + 2) * D + j];
    }
    c += a;
    cx += fmaf(a, xp[0], ax);
    cy += fmaf(a, xp[1], ay);
  }
  red[0][grp][j] = c;
  red[1][grp][j] = cx;
  red[2][grp][j] = cy;
  __syncthreads();
  if (grp == 0) {
    c = cx = cy = 0.0f;
#pragma unroll
    for (int g = 0; g < kL1Groups; ++g) {
      c += red[0][g][j];
      cx += red[1][g][j];
      cy += red[2][g][j];
    }
    out[b * D + j] = c;
    out[(B + b) * D + j] = cx;
    out[(2 * B + b) * D + j] = cy;
  }
}

// grad W1g[j][k] = sum_b (c0[b][j] + c1[b][j]) G[b][k]; grad b1 = sum_b c[b][j]
// and grad W1x[j] = (sum_b cx[b][j], sum_b cy[b][j]), c = c0 + c1 from the two
// passes. Two deterministic stages: workgroup (g, ch) sums the conditions of
// chunk ch (L consecutive ones, staged through LDS 64 at a time, ascending)
// for rows j in [8 g, 8 g + 8) into part[ch][j][0..130] (128 W1g columns,
// then x, y, bias); layer1_sum_kernel adds the chunk partials in chunk order.
constexpr int kL1Rows = 8, kL1Chunk = 64;   // kL1MaxChunks: mf_internal.h

// The first layer's input columns are the boundary vector (ncols = 128) or,
// for the convolutional network, the embedding (ncols = 128 C); blockIdx.z
// takes 128 of them, and a partial row holds ncols + 3 values.
template <int D>
__global__ __launch_bounds__(256) void layer1_part_kernel(const float* __restrict__ l1a,
                                                          const float* __restrict__ l1b,
                                                          const float* __restrict__ G, int ncols, int64_t B,
                                                          int64_t L, float* __restrict__ part) {
  __shared__ float gs[kL1Chunk][128];
  __shared__ float ls[3][kL1Chunk][kL1Rows];   // c, cx, cy of the rows
  const int j0 = blockIdx.x * kL1Rows;
  const int64_t ch = blockIdx.y;
  const int col0 = 128 * blockIdx.z, pw = ncols + 3;
  const int64_t b_begin = ch * L, b_end = std::min<int64_t>(B, b_begin + L);
  const int k = threadIdx.x & 127, js = threadIdx.x >> 7;   // rows j0 + js + 2 i, i < 4
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  float sacc = 0.0f;   // threads < 24: sum type t = tid / 8 (x, y, bias) of row j0 + tid % 8
  for (int64_t b0 = b_begin; b0 < b_end; b0 += kL1Chunk) {
    const int nb = (int)std::min<int64_t>(kL1Chunk, b_end - b0);
    for (int idx = threadIdx.x; idx < kL1Chunk * 128; idx += 256) {
      const int bb = idx >> 7, kk = idx & 127;
      gs[bb][kk] = bb < nb ? G[(b0 + bb) * ncols + col0 + kk] : 0.0f;
    }
    for (int idx = threadIdx.x; idx < 3 * kL1Chunk * kL1Rows; idx += 256) {
      const int t = idx / (kL1Chunk * kL1Rows), r = idx - t * (kL1Chunk * kL1Rows);
      const int bb = r / kL1Rows, jj = r - bb * kL1Rows;
      const int64_t o = ((int64_t)t * B + b0 + bb) * D + j0 + jj;
      ls[t][bb][jj] = bb < nb ? l1a[o] + l1b[o] : 0.0f;
    }
    __syncthreads();
    for (int bb = 0; bb < nb; ++bb) {
      const float g = gs[bb][k];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = fmaf(ls[0][bb][js + 2 * i], g, acc[i]);
    }
    if (blockIdx.z == 0 && threadIdx.x < 3 * kL1Rows) {
      const int t = threadIdx.x / kL1Rows, jj = threadIdx.x - t * kL1Rows;
      const int src = t == 2 ? 0 : t + 1;   // x <- cx, y <- cy, bias <- c
      for (int bb = 0; bb < nb; ++bb) sacc += ls[src][bb][jj];
    }
    __syncthreads();
  }
  float* pp = part + (ch * D + j0) * pw;
#pragma unroll
  for (int i = 0; i < 4; ++i) pp[(js + 2 * i) * pw + col0 + k] = acc[i];
  if (blockIdx.z == 0 && threadIdx.x < 3 * kL1Rows) {
    const int t = threadIdx.x / kL1Rows, jj = threadIdx.x - t * kL1Rows;
    pp[jj * pw + ncols + t] = sacc;
  }
}

// W1 (D rows of ncols + 2: the input columns, then x and y) at w1_off, b1
// after it.
template <int D>
__global__ __launch_bounds__(256) void layer1_sum_kernel(const float* __restrict__ part, int n_chunks, int ncols,
                                                         int64_t w1_off, float* __restrict__ grad) {
  const int pw = ncols + 3;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= D * pw) return;
  const int j = idx / pw, c = idx - j * pw;
  float v = 0.0f;
  for (int ch = 0; ch < n_chunks; ++ch) v += part[(int64_t)ch * D * pw + idx];
  if (c < ncols + 2) grad[w1_off + (int64_t)j * (ncols + 2) + c] = v;   // W1 input columns, then x and y
  else grad[w1_off + (int64_t)D * (ncols + 2) + j] = v;                 // b1
}

// Output-layer gradient and the two losses from the per-wave partials:
// eight threads per element each sum every eighth wave's partial, and the
// eight sums are added in order.
template <int D>
__global__ __launch_bounds__(256) void output_grad_kernel(const float* __restrict__ op_data,
                                                          const float* __restrict__ op_col,
                                                          float inv_data, float inv_col, int64_t off_w5,
                                                          float* __restrict__ grad,
                                                          float* __restrict__ loss) {
  constexpr int EPB = 256 / kReduceGroups;
  __shared__ float sh[2][kReduceGroups][EPB];
  const int e = threadIdx.x % EPB, g = threadIdx.x / EPB;
  const int j = blockIdx.x * EPB + e;
  float s0 = 0.0f, s1 = 0.0f;
  if (j < D + 2) {
#pragma unroll 8
    for (int w = g; w < kOutWaves; w += kReduceGroups) {
      s0 += op_data[(int64_t)w * (D + 2) + j];
      s1 += op_col[(int64_t)w * (D + 2) + j];
    }
  }
  sh[0][g][e] = s0;
  sh[1][g][e] = s1;
  __syncthreads();
  if (g == 0 && j < D + 2) {
    float t0 = 0.0f, t1 = 0.0f;
#pragma unroll
    for (int q = 0; q < kReduceGroups; ++q) {
      t0 += sh[0][q][e];
      t1 += sh[1][q][e];
    }
    if (j <= D) grad[off_w5 + j] = t0 + t1;
    else {
      const float ld = t0 * inv_data, lp = t1 * inv_col;
      loss[0] = ld;
      loss[1] = lp;
      loss[2] = ld + lp;
    }
  }
}

// Adam with bias correction; omb1 = 1 - beta1 and omb2 = 1 - beta2 are
// formed in double on the host.
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float omb1,
                            float b2, float omb2, float eps, float bc1, float bc2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mhat = mi / bc1, vhat = vi / bc2;
    p[i] -= lr * mhat / (sqrtf(vhat) + eps);
  }
}

// Forward-only output for sdnet_forward with derivatives: one wave per point.
template <int D>
__global__ __launch_bounds__(256) void forward_derivs_kernel(const float* __restrict__ Z4,
                                                             const float* __restrict__ w5,
                                                             const float* __restrict__ b5,
                                                             int64_t n_rows, float* __restrict__ U,
                                                             float* __restrict__ dU,
                                                             float* __restrict__ lapU) {
  constexpr int NJ = D / 64;
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = gw; r < n_rows; r += nw) {
    float p[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
      const float w = w5[lane + 64 * t];
#pragma unroll
      for (int sgm = 0; sgm < 4; ++sgm) p[sgm] = fmaf(w, Z4[(4 * r + sgm) * D + lane + 64 * t], p[sgm]);
    }
#pragma unroll
    for (int sgm = 0; sgm < 4; ++sgm)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) p[sgm] += __shfl_xor(p[sgm], off);
    if (lane == 0) {
      if (U) U[r] = p[0] + b5[0];
      if (dU) {
        dU[2 * r] = p[1];
        dU[2 * r + 1] = p[2];
      }
      if (lapU) lapU[r] = p[3];
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side drivers
// ---------------------------------------------------------------------------
static int grid_for(int64_t n, int block, int cap = 8192) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, cap));
}

// skip_last_xy: the last layer's d/dx and d/dy streams are not written (the
// training loss reads only its value and Laplacian streams).
// Persistent grid of the Taylor GEMM: four workgroups per CU (the LDS tile
// allows four), at most one per tile.
static unsigned gemm_grid(int64_t n_tiles) {
  static int n_cu = 0;
  if (n_cu == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || n < 1)
      n = 256;
    n_cu = n;
  }
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_tiles, (int64_t)4 * n_cu));
}

template <int D, int ACT = ACT_TANH>
static hipError_t run_taylor_forward(const NetPtrs& net, const float* C, const float* X, int x_per_bc,
                                     int64_t rows_per_bc, int64_t n_rows, int S, float* const Z[4],
                                     float* const Sv[4], bool skip_last_xy, hipStream_t s) {
  const int64_t n_srows = S * n_rows;
  if (S == 4)
    hipLaunchKernelGGL((fwd_layer1_kernel<D, 4, ACT>), dim3(grid_for(n_rows * D, 256)), dim3(256), 0, s, C,
                       X, x_per_bc, rows_per_bc, n_rows, net.w1x, Z[0], ACT == ACT_GELU ? Sv[0] : nullptr);
  else
    hipLaunchKernelGGL((fwd_layer1_kernel<D, 1, ACT>), dim3(grid_for(n_rows * D, 256)), dim3(256), 0, s, C,
                       X, x_per_bc, rows_per_bc, n_rows, net.w1x, Z[0], ACT == ACT_GELU ? Sv[0] : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned blocks = gemm_grid((n_srows + 63) / 64);
  for (int l = 0; l < 3; ++l) {
    const floatx4* w = static_cast<const floatx4*>(net.wh) + (size_t)l * D * D / 4;
    if (S == 4)
      hipLaunchKernelGGL((taylor_gemm_kernel<D, 4, 0, ACT>), dim3(blocks), dim3(2 * D), 0, s, Z[l], w,
                         net.bh + l * D, nullptr, Z[l + 1], Sv[l + 1], n_srows, (skip_last_xy && l == 2) ? 1 : 0);
    else
      hipLaunchKernelGGL((taylor_gemm_kernel<D, 1, 0, ACT>), dim3(blocks), dim3(2 * D), 0, s, Z[l], w,
                         net.bh + l * D, nullptr, Z[l + 1], ACT == ACT_GELU ? Sv[l + 1] : nullptr, n_srows, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int D, int ACT>
static hipError_t run_pass(const NetPtrs& net, const float* whT, const TrainBuffers& tb, int64_t off_w2,
                           const float* C, const float* X, int x_per_bc, int64_t rows_per_bc,
                           int64_t B, int S, const float* target, float* grad, float* opart,
                           float* l1out, bool accumulate, hipStream_t s) {
  const int64_t n_rows = B * rows_per_bc;
  const int64_t n_srows = S * n_rows;
  float* const* Z = tb.Z;
  // value-only rows keep z in Z for tanh; GELU saves its pre-activations
  float* const* Sv = (S == 4 || ACT == ACT_GELU) ? tb.Sv : tb.Z;
  hipError_t e = run_taylor_forward<D, ACT>(net, C, X, x_per_bc, rows_per_bc, n_rows, S, Z, Sv, true, s);
  if (e != hipSuccess) return e;
  const float inv_n = 1.0f / (float)n_rows;
  if (S == 4)
    hipLaunchKernelGGL((output_loss_kernel<D, 4, ACT>), dim3(kOutWaves / 4), dim3(256), 0, s, Z[3], Sv[3],
                       net.w5, net.b5, target, n_rows, inv_n, tb.Ab[0], opart);
  else
    hipLaunchKernelGGL((output_loss_kernel<D, 1, ACT>), dim3(kOutWaves / 4), dim3(256), 0, s, Z[3], Sv[3],
                       net.w5, net.b5, target, n_rows, inv_n, tb.Ab[0], opart);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  const int64_t lstride = (int64_t)D * D + D;
  const int64_t n_tiles = (n_srows + 63) / 64;
  const int64_t groups = std::min<int64_t>(n_tiles, kBwdGroups);
  int cur = 0;
  for (int l = 2; l >= 0; --l) {           // hidden layer l+2, input Z[l]
    float* Ab = tb.Ab[cur];
    const floatx4* wT = reinterpret_cast<const floatx4*>(whT) + (size_t)l * D * D / 4;
    // layer 1's stream derivatives are W1x and 0 for every row: not stored
    // (GELU keeps layer 1's pre-activations in Sv[0])
    const bool l1 = S == 4 && l == 0;
    const float* svl = (l1 && ACT != ACT_GELU) ? nullptr : Sv[l];
    float* out = tb.Ab[cur ^ 1];
    if constexpr (D <= 128) {
      if (l1)
        hipLaunchKernelGGL((taylor_bwd_split_kernel<D, 4, true, ACT>), dim3((unsigned)groups), dim3(4 * D), 0, s, Ab,
                           Z[l], wT, svl, net.w1x, out, n_srows, tb.wpart, tb.bpart);
      else if (S == 4)
        hipLaunchKernelGGL((taylor_bwd_split_kernel<D, 4, false, ACT>), dim3((unsigned)groups), dim3(4 * D), 0, s, Ab,
                           Z[l], wT, svl, net.w1x, out, n_srows, tb.wpart, tb.bpart);
      else
        hipLaunchKernelGGL((taylor_bwd_split_kernel<D, 1, false, ACT>), dim3((unsigned)groups), dim3(4 * D), 0, s, Ab,
                           Z[l], wT, svl, net.w1x, out, n_srows, tb.wpart, tb.bpart);
    } else {
      if (l1)
        hipLaunchKernelGGL((taylor_bwd_seq_kernel<D, 4, true, ACT>), dim3((unsigned)groups), dim3(2 * D), 0, s, Ab,
                           Z[l], wT, svl, net.w1x, out, n_srows, tb.wpart, tb.bpart);
      else if (S == 4)
        hipLaunchKernelGGL((taylor_bwd_seq_kernel<D, 4, false, ACT>), dim3((unsigned)groups), dim3(2 * D), 0, s, Ab,
                           Z[l], wT, svl, net.w1x, out, n_srows, tb.wpart, tb.bpart);
      else
        hipLaunchKernelGGL((taylor_bwd_seq_kernel<D, 1, false, ACT>), dim3((unsigned)groups), dim3(2 * D), 0, s, Ab,
                           Z[l], wT, svl, net.w1x, out, n_srows, tb.wpart, tb.bpart);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float* gW = grad + off_w2 + l * lstride;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid_for((int64_t)D * D, 256 / kReduceGroups)), dim3(256), 0, s,
                       tb.wpart, groups, (int64_t)D * D, (int64_t)D * D, gW, accumulate ? 1 : 0);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid_for(D, 256 / kReduceGroups)), dim3(256), 0, s, tb.bpart,
                       groups, (int64_t)D, (int64_t)D, gW + (int64_t)D * D, accumulate ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cur ^= 1;
  }
  if (S == 4)
    hipLaunchKernelGGL((layer1_reduce_kernel<D, 4>), dim3((unsigned)B), dim3(kL1Groups * D), 0, s, tb.Ab[cur], X,
                       x_per_bc, rows_per_bc, B, l1out);
  else
    hipLaunchKernelGGL((layer1_reduce_kernel<D, 1>), dim3((unsigned)B), dim3(kL1Groups * D), 0, s, tb.Ab[cur], X,
                       x_per_bc, rows_per_bc, B, l1out);
  return hipGetLastError();
}

hipError_t launch_prepare_wT(const float* params, int64_t off_w2, int width, float* whT, hipStream_t s) {
  hipLaunchKernelGGL(prepare_wT_kernel, dim3(256), dim3(256), 0, s, params, off_w2, width, whT);
  return hipGetLastError();
}

template <int D, int ACT>
static hipError_t train_step_d(const TrainNet& tn, const NetPtrs& net, const float* whT, const TrainBuffers& tb,
                               const float* G, int64_t B, const float* Xd, int64_t nd, int xd_per_bc,
                               const float* Yd, const float* Xc, int64_t nc, float* grad, float* loss,
                               hipStream_t s) {
  hipError_t e = ACT == ACT_GELU
                     ? launch_embed_project(tn.params, D, tn.channels, net, G, B, nullptr, 0, 0, 0, 0, tb.C, s)
                     : launch_projection(net, D, G, B, tb.C, s);
  if (e != hipSuccess) return e;
  // Alg. 1 step 1: data points, value stream only; the targets are Yd, or
  // the boundary vector itself (boundary match at the 128 perimeter nodes).
  e = run_pass<D, ACT>(net, whT, tb, tn.off_w2, tb.C, Xd, xd_per_bc, nd, B, 1, Yd ? Yd : G, grad, tb.opart[0],
                       tb.l1[0], false, s);
  if (e != hipSuccess) return e;
  // Alg. 1 step 2: collocation points, four streams; accumulate.
  e = run_pass<D, ACT>(net, whT, tb, tn.off_w2, tb.C, Xc, 1, nc, B, 4, nullptr, grad, tb.opart[1], tb.l1[1], true,
                       s);
  if (e != hipSuccess) return e;
  // first-layer gradient over its input columns (the boundary vector, or the
  // embedding, recomputed per condition); the weight-gradient partials
  // (already reduced into grad by both passes) hold its chunk partials
  const float* cols = G;
  if (ACT == ACT_GELU) {
    e = launch_embed_grad(tn.params, D, tn.channels, tn.off_w1, G, B, nullptr, nullptr, tb.emb, nullptr, s);
    if (e != hipSuccess) return e;
    cols = tb.emb;
  }
  const int64_t L = std::max<int64_t>(kL1Chunk, ((B + kL1MaxChunks - 1) / kL1MaxChunks + kL1Chunk - 1) /
                                                    kL1Chunk * kL1Chunk);
  const int n_chunks = (int)((B + L - 1) / L);
  hipLaunchKernelGGL((layer1_part_kernel<D>), dim3(D / kL1Rows, n_chunks, tn.n_in / 128), dim3(256), 0, s, tb.l1[0],
                     tb.l1[1], cols, tn.n_in, B, L, tb.wpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((layer1_sum_kernel<D>), dim3((D * (tn.n_in + 3) + 255) / 256), dim3(256), 0, s, tb.wpart,
                     n_chunks, tn.n_in, tn.off_w1, grad);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ACT == ACT_GELU) {   // the embedding's convolutions, from the first layer's per-condition sums
    e = launch_embed_grad(tn.params, D, tn.channels, tn.off_w1, G, B, tb.l1[0], tb.l1[1], nullptr, tb.cpart, s);
    if (e != hipSuccess) return e;
    const int64_t n_conv = tn.off_w1;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid_for(n_conv, 256 / kReduceGroups)), dim3(256), 0, s, tb.cpart,
                       B, n_conv, n_conv, grad, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL((output_grad_kernel<D>), dim3((D + 2 + 256 / kReduceGroups - 1) / (256 / kReduceGroups)),
                     dim3(256), 0, s, tb.opart[0], tb.opart[1],
                     1.0f / (float)(B * nd), 1.0f / (float)(B * nc), tn.off_w5, grad, loss);
  return hipGetLastError();
}

hipError_t launch_train_grad(const TrainNet& tn, const NetPtrs& net, int width, const float* whT,
                             const TrainBuffers& tb, const float* G, int64_t B, const float* Xd, int64_t nd,
                             int xd_per_bc, const float* Yd, const float* Xc, int64_t nc, float* grad, float* loss,
                             hipStream_t s) {
  if (tn.channels > 0)
    return width == 256 ? train_step_d<256, ACT_GELU>(tn, net, whT, tb, G, B, Xd, nd, xd_per_bc, Yd, Xc, nc, grad,
                                                      loss, s)
                        : train_step_d<128, ACT_GELU>(tn, net, whT, tb, G, B, Xd, nd, xd_per_bc, Yd, Xc, nc, grad,
                                                      loss, s);
  return width == 256 ? train_step_d<256, ACT_TANH>(tn, net, whT, tb, G, B, Xd, nd, xd_per_bc, Yd, Xc, nc, grad,
                                                    loss, s)
                      : train_step_d<128, ACT_TANH>(tn, net, whT, tb, G, B, Xd, nd, xd_per_bc, Yd, Xc, nc, grad,
                                                    loss, s);
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, double lr, double b1,
                       double b2, double eps, int64_t step, hipStream_t s) {
  const double bc1 = 1.0 - pow(b1, (double)step), bc2 = 1.0 - pow(b2, (double)step);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, p, m, v, g, n,
                     (float)lr, (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps,
                     (float)bc1, (float)bc2);
  return hipGetLastError();
}

// The GELU network's value stream saving each layer's pre-activations in Sv
// (for its reverse pass): first layer from C [n_bc][D] and shared points
// X [T][2], then the three hidden layers.
hipError_t launch_value_forward_gelu_saved(const NetPtrs& net, int width, const float* C, const float* X, int64_t T,
                                           int64_t n_bc, float* const Z[4], float* const Sv[4], hipStream_t s) {
  return width == 256 ? run_taylor_forward<256, ACT_GELU>(net, C, X, 0, T, n_bc * T, 1, Z, Sv, false, s)
                      : run_taylor_forward<128, ACT_GELU>(net, C, X, 0, T, n_bc * T, 1, Z, Sv, false, s);
}

// Value stream only: first layer from C [n_bc][D] and shared points X [T][2],
// then the three hidden layers; Z[l] receives layer l+1's activations.
hipError_t launch_value_forward(const NetPtrs& net, int width, const float* C, const float* X, int64_t T,
                                int64_t n_bc, float* const Z[4], hipStream_t s) {
  float* Sv[4] = {nullptr, nullptr, nullptr, nullptr};
  return width == 256 ? run_taylor_forward<256>(net, C, X, 0, T, n_bc * T, 1, Z, Sv, false, s)
                      : run_taylor_forward<128>(net, C, X, 0, T, n_bc * T, 1, Z, Sv, false, s);
}

// Value-stream reverse pass from ab4 in Ab[0] down to ab1, then per-condition
// sums c[b][j] = sum_t ab1 (first of the three [n_bc][D] blocks of csum).
template <int D>
static hipError_t value_backward_d(const float* whT, float* const Z[4], float* const Sv[4], float* const Ab[2],
                                   int64_t n_rows, const float* X, int64_t n_bc, int64_t T, float* csum,
                                   hipStream_t s) {
  int cur = 0;
  const unsigned blocks = gemm_grid((n_rows + 63) / 64);
  for (int l = 2; l >= 0; --l) {
    const floatx4* wT = reinterpret_cast<const floatx4*>(whT) + (size_t)l * D * D / 4;
    if (Sv)   // GELU: the reverse rule needs the saved pre-activations
      hipLaunchKernelGGL((taylor_gemm_kernel<D, 1, 1, ACT_GELU>), dim3(blocks), dim3(2 * D), 0, s, Ab[cur], wT,
                         nullptr, Sv[l], Ab[cur ^ 1], nullptr, n_rows, 0);
    else
      hipLaunchKernelGGL((taylor_gemm_kernel<D, 1, 1>), dim3(blocks), dim3(2 * D), 0, s, Ab[cur], wT, nullptr,
                         Z[l], Ab[cur ^ 1], nullptr, n_rows, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  hipLaunchKernelGGL((layer1_reduce_kernel<D, 1>), dim3((unsigned)n_bc), dim3(kL1Groups * D), 0, s, Ab[cur], X, 0, T, n_bc,
                     csum);
  return hipGetLastError();
}

hipError_t launch_value_backward(const float* whT, int width, float* const Z[4], float* const Sv[4],
                                 float* const Ab[2], int64_t n_rows, const float* X, int64_t n_bc, int64_t T,
                                 float* csum, hipStream_t s) {
  return width == 256 ? value_backward_d<256>(whT, Z, Sv, Ab, n_rows, X, n_bc, T, csum, s)
                      : value_backward_d<128>(whT, Z, Sv, Ab, n_rows, X, n_bc, T, csum, s);
}

// Value stream of either activation, rows_per_bc points per condition (X
// shared [rows_per_bc][2] or per row [n_rows][2]); Z[l] receives layer
// l+1's activations (buffers may alternate: layer l reads only Z[l - 1]).
hipError_t launch_value_forward_act(const NetPtrs& net, int width, int act, const float* C, const float* X,
                                    int x_per_bc, int64_t rows_per_bc, int64_t n_rows, float* const Z[4],
                                    hipStream_t s) {
  float* Sv[4] = {nullptr, nullptr, nullptr, nullptr};
  if (act == ACT_GELU)
    return width == 256 ? run_taylor_forward<256, ACT_GELU>(net, C, X, x_per_bc, rows_per_bc, n_rows, 1, Z, Sv, false, s)
                        : run_taylor_forward<128, ACT_GELU>(net, C, X, x_per_bc, rows_per_bc, n_rows, 1, Z, Sv, false, s);
  return width == 256 ? run_taylor_forward<256>(net, C, X, x_per_bc, rows_per_bc, n_rows, 1, Z, Sv, false, s)
                      : run_taylor_forward<128>(net, C, X, x_per_bc, rows_per_bc, n_rows, 1, Z, Sv, false, s);
}

hipError_t launch_forward_derivs(const NetPtrs& net, int width, int act, const float* C, const float* X,
                                 int x_per_bc, int64_t n_bc, int64_t n_pts, float* Z0, float* Z1,
                                 float* U, float* dU, float* lapU, hipStream_t s) {
  float* Z[4] = {Z0, Z1, Z0, Z1};
  float* Sv[4] = {nullptr, nullptr, nullptr, nullptr};
  const int64_t n_rows = n_bc * n_pts;
  hipError_t e;
  if (act == ACT_GELU)
    e = width == 256 ? run_taylor_forward<256, ACT_GELU>(net, C, X, x_per_bc, n_pts, n_rows, 4, Z, Sv, false, s)
                     : run_taylor_forward<128, ACT_GELU>(net, C, X, x_per_bc, n_pts, n_rows, 4, Z, Sv, false, s);
  else
    e = width == 256 ? run_taylor_forward<256>(net, C, X, x_per_bc, n_pts, n_rows, 4, Z, Sv, false, s)
                     : run_taylor_forward<128>(net, C, X, x_per_bc, n_pts, n_rows, 4, Z, Sv, false, s);
  if (e != hipSuccess) return e;
  const int blocks = grid_for(n_rows, 4, 4096);
  if (width == 256)
    hipLaunchKernelGGL((forward_derivs_kernel<256>), dim3(blocks), dim3(256), 0, s, Z1, net.w5, net.b5,
                       n_rows, U, dU, lapU);
  else
    hipLaunchKernelGGL((forward_derivs_kernel<128>), dim3(blocks), dim3(256), 0, s, Z1, net.w5, net.b5,
                       n_rows, U, dU, lapU);
  return hipGetLastError();
}

}  // namespace mf

// Kernels of the Mosaic Flow sweep on gfx950.
//
// The hot kernel is `tile_kernel`: one workgroup takes R consecutive rows of
// a colour phase, a row being one (placement, target) pair, and runs the
// whole SDNet on them without leaving the CU:
//   1. gather the 128 boundary values of each placement the tile touches
//      (Sec. 4.1: same-colour placements are independent, so the phase is a
//      pure function of the field before it);
//   2. boundary projection W1g g + b1 once per placement (input-split first
//      layer, Eq. 8) and the per-row coordinate term W1x (x, y), then tanh;
//   3. three d x d hidden layers on MFMA, activations resident in LDS, the
//      weights streamed from L2 in the MFMA operand order prepared once per
//      call;
//   4. the scalar output layer, and the store of the prediction into the
//      field (sweep) or the overlap-averaging accumulation (assembly, Alg. 2).
// Rows from neighbouring placements share a tile, so nothing is padded to
// the 61 or 961 targets of a placement.
#include <algorithm>

#include "mf_device.h"
#include "mf_internal.h"

namespace mf {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Network preparation: copy the flat parameters into the kernels' layouts.
// Hidden matrices, per layer:
//   fp32: [cb = d/32][kg = d/8][lane 64][4], lane l, element e holds
//         W[32 cb + (l & 31)][8 kg + 4 (l >> 5) + e]
//   bf16: [cb = d/32][kg = d/16][lane 64][8], lane l, element e holds
//         W[32 cb + (l & 31)][16 kg + 8 (l >> 5) + e]
// so that one wave's B operand for one k-group is 1 KiB of contiguous memory.
// ---------------------------------------------------------------------------
// n_in: columns of W1 before the (x, y) columns: 128 boundary values, or the
// 128 C values of a convolutional embedding (then params points at W1, past
// the convolutions, and w1gT is filled by prepare_w1eT_kernel instead).
__global__ void prepare_net_kernel(const float* __restrict__ params, int d, int prec, int n_in,
                                   float* __restrict__ w1gT, uint16_t* __restrict__ w1gb, float* __restrict__ w1x,
                                   float* __restrict__ b1, void* __restrict__ wh,
                                   float* __restrict__ bh, float* __restrict__ w5,
                                   float* __restrict__ b5) {
  const int64_t ld1 = n_in + 2;   // row length of W1
  const int64_t off_b1 = (int64_t)d * ld1;
  const int64_t off_w2 = off_b1 + d;
  const int64_t lstride = (int64_t)d * d + d;
  const int64_t off_w5 = off_w2 + 3 * lstride;
  const int64_t off_b5 = off_w5 + d;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;

  for (int64_t idx = tid; n_in == 128 && idx < 128 * (int64_t)d; idx += nthr) {
    const int64_t k = idx / d, n = idx - k * d;
    w1gT[idx] = params[n * 130 + k];
    if (prec != MF_FP32) {
      // 16-bit W1g in MFMA operand order, in the precision of the phase
      // [cb = d/32][kg = 8][lane 64][8]: lane l, element e holds
      // W1[32 cb + (l & 31)][16 kg + 8 (l >> 5) + e]
      const int e = (int)(idx & 7), lane = (int)((idx >> 3) & 63);
      const int64_t rest = idx >> 9;
      const int kg = (int)(rest % 8), cb = (int)(rest / 8);
      const float wv = params[(int64_t)(32 * cb + (lane & 31)) * 130 + 16 * kg + 8 * (lane >> 5) + e];
      w1gb[idx] = prec == MF_FP16 ? f16_bits(wv) : bf16_bits(wv);
    }
  }
  for (int64_t n = tid; n < d; n += nthr) {
    w1x[2 * n] = params[n * ld1 + n_in];
    w1x[2 * n + 1] = params[n * ld1 + n_in + 1];
    b1[n] = params[off_b1 + n];
    w5[n] = params[off_w5 + n];
    for (int l = 0; l < 3; ++l) bh[l * d + n] = params[off_w2 + l * lstride + (int64_t)d * d + n];
  }
  if (tid == 0) {
    // b5 and, for the sweep kernel's output layer, b5 + sum(w5) (summed in
    // index order)
    float sw = params[off_b5];
    for (int n = 0; n < d; ++n) sw += params[off_w5 + n];
    b5[0] = params[off_b5];
    b5[1] = sw;
  }

  const int64_t dd = (int64_t)d * d;
  for (int64_t idx = tid; idx < 3 * dd; idx += nthr) {
    const int l = (int)(idx / dd);
    const int64_t r = idx - l * dd;
    int j, k;
    if (prec == MF_FP32) {
      const int e = r & 3, lane = (r >> 2) & 63;
      const int64_t rest = r >> 8;
      const int kg = (int)(rest % (d / 8)), cb = (int)(rest / (d / 8));
      j = 32 * cb + (lane & 31);
      k = 8 * kg + 4 * (lane >> 5) + e;
      static_cast<float*>(wh)[idx] = params[off_w2 + l * lstride + (int64_t)j * d + k];
    } else {
      const int e = r & 7, lane = (r >> 3) & 63;
      const int64_t rest = r >> 9;
      const int kg = (int)(rest % (d / 16)), cb = (int)(rest / (d / 16));
      j = 32 * cb + (lane & 31);
      k = 16 * kg + 8 * (lane >> 5) + e;
      const float wv = params[off_w2 + l * lstride + (int64_t)j * d + k];
      static_cast<uint16_t*>(wh)[idx] = prec == MF_FP16 ? f16_bits(wv) : bf16_bits(wv);
    }
  }
}

hipError_t launch_prepare_net(const float* params, int width, int prec, const NetLayout& L,
                              void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  hipLaunchKernelGGL(prepare_net_kernel, dim3(256), dim3(256), 0, s, params, width, prec, 128,
                     reinterpret_cast<float*>(base + L.w1gT), reinterpret_cast<uint16_t*>(base + L.w1gb),
                     reinterpret_cast<float*>(base + L.w1x),
                     reinterpret_cast<float*>(base + L.b1), static_cast<void*>(base + L.wh),
                     reinterpret_cast<float*>(base + L.bh), reinterpret_cast<float*>(base + L.w5),
                     reinterpret_cast<float*>(base + L.b5));
  return hipGetLastError();
}

hipError_t launch_prepare_net_embed(const float* params, int width, int C, const NetLayout& L, void* ws,
                                    hipStream_t s) {
  char* base = static_cast<char*>(ws);
  hipLaunchKernelGGL(prepare_net_kernel, dim3(256), dim3(256), 0, s, params + embed_param_offset(C), width,
                     (int)MF_FP32, C * kNB, reinterpret_cast<float*>(base + L.w1gT), nullptr,
                     reinterpret_cast<float*>(base + L.w1x), reinterpret_cast<float*>(base + L.b1),
                     static_cast<void*>(base + L.wh), reinterpret_cast<float*>(base + L.bh),
                     reinterpret_cast<float*>(base + L.w5), reinterpret_cast<float*>(base + L.b5));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_prepare_w1eT(params, width, C, reinterpret_cast<float*>(base + L.w1gT), s);
}

// ---------------------------------------------------------------------------
// The fused tile kernel.
// ---------------------------------------------------------------------------
enum { SRC_GATHER = 0, SRC_C = 1 };
enum { OUT_STORE = 0, OUT_ACCUM = 1, OUT_LINEAR = 2 };

struct TileArgs {
  NetPtrs net;
  // SRC_GATHER: the field of one domain and the colour of the phase
  const float* u_in;
  float* u_out;
  int64_t pitch;
  int ux, uy, colour;
  // SRC_C: precomputed projections C [n_bc][d] (b1 included) and points
  const float* C;
  const float* X;
  int64_t n_pts;
  int x_per_bc;
  float* U;
  int64_t total_rows;
  int64_t block0;   // first tile of this launch (large phases take several launches)
};

template <int PREC> struct HType { typedef float T; };
template <> struct HType<1> { typedef uint16_t T; };
template <> struct HType<2> { typedef uint16_t T; };

// MFMA on one k group of a d x d layer. The prepared weights are the A
// operand (rows = output units j) and the activations the B operand (columns
// = points i), so a lane's accumulator registers 4g .. 4g + 3 hold four
// consecutive units of one point: the epilogue converts and stores them as
// one 16-byte (fp32) or 8-byte (bf16) vector. Inside a k group lane l feeds
// the same k indices to both operands (fp32: k = 4 (l >> 5) + e at step e;
// bf16: k = 8 (l >> 5) + e), which is what the prepared layout holds.
template <int PREC> struct Mma;
template <> struct Mma<0> {
  typedef floatx4 T;
  static constexpr int K = 8;
  template <int N>
  static __device__ __forceinline__ void run(const T& w, const T (&h)[N], floatx16 (&c)[N]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int n = 0; n < N; ++n) c[n] = mfma32x32x2(w[e], h[n][e], c[n]);
  }
};
template <> struct Mma<1> {
  typedef bf16x8 T;
  static constexpr int K = 16;
  static __device__ __forceinline__ floatx16 one(const T& w, const T& h, const floatx16& c) {
    return mfma32x32x16_bf16(w, h, c);
  }
  template <int N>
  static __device__ __forceinline__ void run(const T& w, const T (&h)[N], floatx16 (&c)[N]) {
#pragma unroll
    for (int n = 0; n < N; ++n) c[n] = one(w, h[n], c[n]);
  }
  // two floats -> one register of two operand elements
  static __device__ __forceinline__ uint32_t pack(float a, float b) {
    const bf16x2 p = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, p);
  }
};
// fp16 operands: the same layouts and k order as bf16; three more mantissa
// bits for weights and activations, range +-65504 (activations are k tanh,
// |k tanh| < 2.9; hidden weights must stay below 65504).
template <> struct Mma<2> {
  typedef halfx8 T;
  static constexpr int K = 16;
  static __device__ __forceinline__ floatx16 one(const T& w, const T& h, const floatx16& c) {
    return mfma32x32x16_f16(w, h, c);
  }
  template <int N>
  static __device__ __forceinline__ void run(const T& w, const T (&h)[N], floatx16 (&c)[N]) {
#pragma unroll
    for (int n = 0; n < N; ++n) c[n] = one(w, h[n], c[n]);
  }
  // The values pass through an opaque move: otherwise the compiler folds the
  // tanh's last fma into a mixed-precision fma with fp16 output in some tile
  // forms and not in others, and the tiles would round differently. (A
  // non-volatile move gives the same bits and a 2% faster row-split phase,
  // but the row-split tile then spills 40 bytes per lane.)
  static __device__ __forceinline__ uint32_t pack(float a, float b) {
    asm volatile("" : "+v"(a), "+v"(b));
    const halfx2 p = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, p);
  }
};

template <int PREC>
__device__ __forceinline__ typename Mma<PREC>::T load_op(const void* p) {
  return __builtin_bit_cast(typename Mma<PREC>::T, *static_cast<const u32x4*>(p));
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Four consecutive activations of one row.
template <int PREC>
__device__ __forceinline__ void store4(typename HType<PREC>::T* p, float a, float b, float c, float d) {
  if constexpr (PREC == 0) {
    *reinterpret_cast<floatx4*>(p) = floatx4{a, b, c, d};
  } else {
    *reinterpret_cast<u32x2*>(p) = u32x2{Mma<PREC>::pack(a, b), Mma<PREC>::pack(c, d)};
  }
}

// Activations are stored multiplied by k = 2 log2(e): a layer's accumulator
// then holds k z (its bias is stored as k b too), and
//   k tanh(z) = k - 2 k / (1 + 2^(k z)),
// one exp2, one reciprocal and one fma; the scale costs nothing.
__device__ __forceinline__ float rsig_exp2(float kz) {   // 1 / (1 + e^(2z))
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(kz));
}
__device__ __forceinline__ float ktanh_exp2(float kz) {
  return fmaf(-2.0f * kTwoLog2e, rsig_exp2(kz), kTwoLog2e);
}

// Accumulator of one 32 x 32 block initialised with the (scaled) bias of its
// units; `b` points at unit col0 + 4 (lane >> 5).
__device__ __forceinline__ floatx16 bias_acc(const float* b) {
  floatx16 a;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const floatx4 v = *reinterpret_cast<const floatx4*>(b + 8 * g);
#pragma unroll
    for (int e = 0; e < 4; ++e) a[4 * g + e] = v[e];
  }
  return a;
}

// k tanh of one finished block, written to the activation rows in place.
template <int PREC>
__device__ __forceinline__ void store_tanh(typename HType<PREC>::T* p, const floatx16& acc) {
#pragma unroll
  for (int g = 0; g < 4; ++g)
    store4<PREC>(p + 8 * g, ktanh_exp2(acc[4 * g]), ktanh_exp2(acc[4 * g + 1]), ktanh_exp2(acc[4 * g + 2]),
                 ktanh_exp2(acc[4 * g + 3]));
}

// Output layer folded into the last hidden layer: with tanh z = 1 - 2 r,
// w5 . tanh(z) = sum(w5) + sum(-2 w5 r); here the second sum over the lane's
// 16 units (`w` holds -2 w5 at unit col0 + 4 (lane >> 5)).
__device__ __forceinline__ float dot_tanh(const floatx16& acc, const float* w) {
  float s = 0.0f;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const floatx4 v = *reinterpret_cast<const floatx4*>(w + 8 * g);
#pragma unroll
    for (int e = 0; e < 4; ++e) s = fmaf(v[e], rsig_exp2(acc[4 * g + e]), s);
  }
  return s;
}

// Partial output of one 32-column block for the 32 points of a row block:
// the two half-waves hold the two halves of the block's units.
__device__ __forceinline__ void put_partial(float* po, float s, int lane) {
  s += __shfl_xor(s, 32);
  if (lane < 32) po[lane] = s;
}

// The wave's CPW-column slice of hidden layer l's prepared weights: D/KK
// MFMA operands per 32 columns. The layer offset is opaque to the optimiser,
// which would otherwise hoist the loads of all three layers (and, in the
// persistent kernel, out of the tile loop) and run out of registers.
template <int D, int PREC, int CPW>
__device__ __forceinline__ const u32x4* wslice(const u32x4* wh, int l, int wave, int lane, int cb) {
  constexpr int KG = D / Mma<PREC>::K, NCB = CPW / 32;
  constexpr int LAYER = D * D / (PREC == 0 ? 4 : 8);   // u32x4 per prepared layer
  int lofs = l * LAYER;
  asm volatile("" : "+s"(lofs));
  return wh + lofs + (wave * NCB + cb) * KG * 64 + lane;
}

template <int D, int PREC, int CPW>
__device__ __forceinline__ void load_wslice(typename Mma<PREC>::T (&wreg)[CPW / 32][D / Mma<PREC>::K],
                                            const u32x4* wh, int l, int wave, int lane) {
#pragma unroll
  for (int cb = 0; cb < CPW / 32; ++cb) {
    const u32x4* wsw = wslice<D, PREC, CPW>(wh, l, wave, lane, cb);
#pragma unroll
    for (int kg = 0; kg < D / Mma<PREC>::K; ++kg)
      wreg[cb][kg] = __builtin_bit_cast(typename Mma<PREC>::T, wsw[kg * 64]);
  }
}

// One hidden layer with the wave's weight slice in registers (`wreg`, loaded
// by the caller). The wave walks the tile's 32-row blocks with one barrier
// per block; the row-block loop is unrolled, so the tanh epilogue of block
// rb - 1 (written back in place: every wave has finished reading those rows
// once it passed the previous barrier) sits in the same basic block as the
// MFMAs of block rb and the scheduler overlaps them. LAST: the output
// layer's dot products instead of activations, no writes to the tile and so
// no barriers. NEXT: during the last row block each weight register is
// reloaded with layer l + 1's operand right after its last MFMA, so the next
// layer's weights arrive while this layer finishes instead of after it.
template <int D, int R, int PREC, int CPW, bool LAST, bool NEXT = false>
__device__ __forceinline__ void layer_wreg(typename HType<PREC>::T* Hs,
                                           typename Mma<PREC>::T (&wreg)[CPW / 32][D / Mma<PREC>::K],
                                           const u32x4* wh, int l, const float* nb, float* po, int lane,
                                           int wave) {
  typedef Mma<PREC> M;
  typedef typename M::T OT;
  constexpr int KK = M::K, KG = D / KK, RB = R / 32, NCB = CPW / 32;
  constexpr int LDH = PREC == 0 ? D + 4 : D + 8;
  const int arow = lane & 31, ahalf = lane >> 5;
  floatx16 acc[2][NCB];
  // one opaque slice pointer per column block (per-load address arithmetic
  // would be hoisted ahead of the MFMAs and spill)
  const u32x4* nsw[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) nsw[cb] = NEXT ? wslice<D, PREC, CPW>(wh, l + 1, wave, lane, cb) : wh;
#pragma unroll
  for (int rb = 0; rb <= RB; ++rb) {
    floatx16(&cur)[NCB] = acc[rb & 1];
    floatx16(&prv)[NCB] = acc[(rb + 1) & 1];
    if (rb < RB) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) cur[cb] = bias_acc(nb + l * D + (wave * NCB + cb) * 32 + 4 * ahalf);
      const typename HType<PREC>::T* ap = Hs + (rb * 32 + arow) * LDH + (KK / 2) * ahalf;
#pragma unroll
      for (int kg = 0; kg < KG; ++kg) {
        const OT h[1] = {load_op<PREC>(ap + kg * KK)};
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          floatx16 c1[1] = {cur[cb]};
          M::template run<1>(wreg[cb][kg], h, c1);
          cur[cb] = c1[0];
          if constexpr (NEXT) {
            if (rb == RB - 1) {
              // MFMAs and memory loads may not cross: the reload stays behind
              // the MFMA that last reads the register
              __builtin_amdgcn_sched_barrier(0x787);
              wreg[cb][kg] = __builtin_bit_cast(OT, nsw[cb][kg * 64]);
            }
          }
        }
      }
    }
    if (rb > 0) {
      const int row = (rb - 1) * 32;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int col = (wave * NCB + cb) * 32;
        if constexpr (!LAST) store_tanh<PREC>(Hs + (row + arow) * LDH + col + 4 * ahalf, prv[cb]);
        else put_partial(po + (col / 32) * R + row, dot_tanh(prv[cb], nb + 3 * D + col + 4 * ahalf), lane);
      }
    }
    if constexpr (!LAST) __syncthreads();
  }
}

// The three hidden layers and the output layer's dot products. `nb` (LDS)
// holds k times the biases of the three hidden layers and then -2 w5; `po` (LDS,
// [D / 32][R]) receives per-32-column partial outputs, summed by the caller
// in a fixed order, so a row's result does not depend on the tile shape.
// WREG: register-resident weights (layer_wreg). Otherwise (fp32 only) the
// weights stream from L2 per k group and serve all row blocks of the tile;
// fewer registers, so more workgroups per CU.
template <int D, int R, int PREC, int CPW, bool WREG>
__device__ __forceinline__ void hidden_and_output(typename HType<PREC>::T* Hs,
                                                  typename Mma<PREC>::T (&wreg)[CPW / 32][D / Mma<PREC>::K],
                                                  const u32x4* wh, const float* nb, float* po, int lane,
                                                  int wave) {
  if constexpr (WREG) {
    // wreg holds layer 0 on entry (loaded by the caller ahead of the first
    // layer, so those loads overlap its tanh work). fp32 reloads the next
    // layer inside the last row block (-1% per phase); in the bf16 tiles,
    // built for 128 VGPRs, the reload spills, so they load between layers.
    constexpr bool RELOAD = PREC == 0;
#pragma unroll 1
    for (int l = 0; l < 2; ++l) {
      if (!RELOAD && l > 0) load_wslice<D, PREC, CPW>(wreg, wh, l, wave, lane);
      layer_wreg<D, R, PREC, CPW, false, RELOAD>(Hs, wreg, wh, l, nb, po, lane, wave);
    }
    if (!RELOAD) load_wslice<D, PREC, CPW>(wreg, wh, 2, wave, lane);
    layer_wreg<D, R, PREC, CPW, true>(Hs, wreg, wh, 2, nb, po, lane, wave);
  } else {
    typedef Mma<PREC> M;
    typedef typename M::T OT;
    constexpr int KK = M::K, KG = D / KK, RB = R / 32;
    constexpr int LDH = PREC == 0 ? D + 4 : D + 8;
    constexpr int LAYER = D * D / (PREC == 0 ? 4 : 8);
    static_assert(PREC == 0 && CPW == 32, "streamed weights: fp32, 32 columns per wave");
    const int arow = lane & 31, ahalf = lane >> 5;
    const int col = wave * 32;
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
      floatx16 acc[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = bias_acc(nb + l * D + col + 4 * ahalf);
      const u32x4* wsw = wh + l * LAYER + wave * KG * 64 + lane;
#pragma unroll 4
      for (int kg = 0; kg < KG; ++kg) {
        const OT w = __builtin_bit_cast(OT, wsw[kg * 64]);
        OT h[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) h[rb] = load_op<PREC>(Hs + (rb * 32 + arow) * LDH + kg * KK + (KK / 2) * ahalf);
        M::template run<RB>(w, h, acc);
      }
      if (l < 2) {
        __syncthreads();   // every wave has finished reading this layer's input
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) store_tanh<PREC>(Hs + (rb * 32 + arow) * LDH + col + 4 * ahalf, acc[rb]);
        __syncthreads();
      } else {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          put_partial(po + wave * R + rb * 32, dot_tanh(acc[rb], nb + 3 * D + col + 4 * ahalf), lane);
      }
    }
  }
  __syncthreads();   // partial outputs complete
}

template <int D, int R, int TMODE, int PREC, int SRC, int OUT, int CPW = 32, bool WREG = true>
__device__ __forceinline__ void tile_body(const TileArgs& A, const int64_t row0) {
  static_assert(CPW == 32 || (CPW == 64 && PREC != 0), "64 columns per wave: 16-bit only");
  constexpr int NTH = (D / CPW) * 64;        // one wave per CPW output columns
  constexpr int T = n_targets<TMODE>();
  constexpr int NPMAX = SRC == SRC_GATHER ? (R - 1) / T + 2 : 1;
  constexpr int LDH = PREC == 0 ? D + 4 : D + 8;   // padded row (elements)
  constexpr int NCOLB = D / 32;
  constexpr int SCR = NPMAX * (kNB + D) > NCOLB * R ? NPMAX * (kNB + D) : NCOLB * R;
  typedef typename HType<PREC>::T HT;

  __shared__ __align__(16) HT Hs[R * LDH];
  __shared__ __align__(16) float scr[SCR];   // boundary values + projections, later partial outputs
  __shared__ __align__(16) floatx4 r_info[R];   // x, y, placement slot (bits), cover weight
  __shared__ __align__(16) float nb[4 * D];   // k b2, k b3, k b4, -2 w5
  __shared__ int64_t r_addr[R];
  __shared__ int64_t r_bc[SRC == SRC_C ? R : 1];
  float* gs = scr;
  float* cs = scr + NPMAX * kNB;
  float* po = scr;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // The network pointers, offset by an opaque zero: in the persistent kernel
  // the optimiser would otherwise hoist every tile-invariant weight load
  // (projection, first layer, hidden layers) out of the tile loop and run
  // out of registers.
  int zero = 0;
  asm volatile("" : "+s"(zero));
  NetPtrs net = A.net;
  net.w1gT += zero;
  net.w1gb = static_cast<const u32x4*>(net.w1gb) + zero;
  net.w1x += zero;
  net.b1 += zero;
  net.bh += zero;
  net.w5 += zero;
  net.wh = static_cast<const u32x4*>(net.wh) + zero;

  for (int i = tid; i < 4 * D; i += NTH) nb[i] = i < 3 * D ? kTwoLog2e * net.bh[i] : -2.0f * net.w5[i - 3 * D];

  // -- rows of this tile -----------------------------------------------------
  int64_t q0 = 0;
  int np = 0;
  if constexpr (SRC == SRC_GATHER) {
    const int64_t last = min(row0 + R, A.total_rows) - 1;
    q0 = row0 / T;
    np = (int)(last / T - q0 + 1);
  }
  for (int rt = tid; rt < R; rt += NTH) {
    const int64_t row = row0 + rt;
    const bool valid = row < A.total_rows;
    const int64_t rr = valid ? row : A.total_rows - 1;
    if constexpr (SRC == SRC_GATHER) {
      const int q = (int)(rr / T), t = (int)(rr - (int64_t)q * T);
      int a, b, ti, tj;
      placement_of(q, A.colour, A.ux, a, b);
      target_local<TMODE>(t, ti, tj);
      const int gi = kHalf * a + ti, gj = kHalf * b + tj;
      r_info[rt] = floatx4{ti * (1.0f / kS), tj * (1.0f / kS), __int_as_float((int)(q - q0)),
                           cover_inv(gi, kS * A.ux) * cover_inv(gj, kS * A.uy)};
      r_addr[rt] = valid ? (int64_t)gj * A.pitch + gi : -1;
    } else {
      const int64_t bc = rr / A.n_pts, pt = rr - bc * A.n_pts;
      const float* xp = A.x_per_bc ? A.X + 2 * rr : A.X + 2 * pt;
      r_info[rt] = floatx4{xp[0], xp[1], 0.0f, 1.0f};
      r_bc[rt] = bc;
      r_addr[rt] = valid ? rr : -1;
    }
  }

  // -- gather + boundary projection (once per placement) --------------------
  // Thread t owns 4 consecutive columns (group t % (D/4)) and a 16-wide slice
  // of k (t / (D/4)); its 16 float4 loads of W1g^T are independent and are
  // issued before the gather, so both latencies overlap.
  constexpr int NG = D / 4, KSL = NTH / NG, KPS = kNB / KSL;
  static_assert(KSL * KPS == kNB, "projection split");
  floatx4 w[KPS];
  const int n4 = tid % NG, ks = tid / NG;
  if constexpr (SRC == SRC_GATHER) {
    if constexpr (PREC == 0) {
#pragma unroll
      for (int i = 0; i < KPS; ++i)
        w[i] = *reinterpret_cast<const floatx4*>(net.w1gT + (ks * KPS + i) * D + 4 * n4);
    }
    for (int idx = tid; idx < np * kNB; idx += NTH) {
      const int s = idx >> 7, k = idx & 127;
      int a, b, bi, bj;
      placement_of((int)(q0 + s), A.colour, A.ux, a, b);
      boundary_local(k, bi, bj);
      gs[idx] = A.u_in[(int64_t)(kHalf * b + bj) * A.pitch + kHalf * a + bi];
    }
    __syncthreads();
    if constexpr (PREC != 0) {
      // 16-bit: W1g G^T on MFMA in the phase's precision. A = the tile's
      // boundary vectors (rows p < np, at most NPMAX <= 8, rounded to the
      // phase's 16-bit type), B = the wave's 32-column slice
      // of W1g in operand order; a lane's accumulator registers 0..3 hold
      // rows 4 (lane >> 5) .. + 3 of its column. The stored projection
      // carries b1 and the factor 2 log2(e) of the tanh.
      static_assert(NPMAX <= 8, "projection rows");
      const int arow = lane & 31, ahalf = lane >> 5;
      constexpr int NCBP = CPW / 32;
#pragma unroll
      for (int cb = 0; cb < NCBP; ++cb) {
        const int col = ((wave % (D / CPW)) * NCBP + cb) * 32 + arow;
        const u32x4* wp = static_cast<const u32x4*>(net.w1gb) + (size_t)((wave % (D / CPW)) * NCBP + cb) * 8 * 64 + lane;
        floatx16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll
        for (int kg = 0; kg < 8; ++kg) {
          typedef typename Mma<PREC>::T PT;
          u32x4 av = u32x4{0u, 0u, 0u, 0u};
          if (arow < np) {
            const floatx4 g0 = *reinterpret_cast<const floatx4*>(&gs[arow * kNB + 16 * kg + 8 * ahalf]);
            const floatx4 g1 = *reinterpret_cast<const floatx4*>(&gs[arow * kNB + 16 * kg + 8 * ahalf + 4]);
            av = u32x4{Mma<PREC>::pack(g0[0], g0[1]), Mma<PREC>::pack(g0[2], g0[3]), Mma<PREC>::pack(g1[0], g1[1]),
                       Mma<PREC>::pack(g1[2], g1[3])};
          }
          acc = Mma<PREC>::one(__builtin_bit_cast(PT, av), __builtin_bit_cast(PT, wp[kg * 64]), acc);
        }
        const float bb = net.b1[col];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int prow = 4 * ahalf + v;
          if (prow < np) cs[prow * D + col] = kTwoLog2e * (acc[v] + bb);
        }
      }
    } else {
    // The k-slice partials go to LDS scratch that aliases the activation tile
    // (not in use yet) and are then summed; the stored projection carries b1
    // and the factor 2 log2(e) of the tanh.
    static_assert((size_t)KSL * NPMAX * D * sizeof(float) <= sizeof(HT) * R * LDH, "projection scratch");
    float* part = reinterpret_cast<float*>(Hs);
    for (int s = 0; s < np; ++s) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int i = 0; i < KPS; ++i) {
        const float g = gs[s * kNB + ks * KPS + i];
        acc[0] = fmaf(w[i][0], g, acc[0]);
        acc[1] = fmaf(w[i][1], g, acc[1]);
        acc[2] = fmaf(w[i][2], g, acc[2]);
        acc[3] = fmaf(w[i][3], g, acc[3]);
      }
      *reinterpret_cast<floatx4*>(&part[(ks * NPMAX + s) * D + 4 * n4]) = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < np * D; idx += NTH) {
      const int s = idx / D, n = idx - s * D;
      float c = 0.0f;
#pragma unroll
      for (int k = 0; k < KSL; ++k) c += part[(k * NPMAX + s) * D + n];
      cs[idx] = kTwoLog2e * (c + net.b1[n]);
    }
    }
  }
  __syncthreads();

  // the first hidden layer's weights are in flight during the first layer
  typename Mma<PREC>::T wreg[CPW / 32][D / Mma<PREC>::K];
  if constexpr (WREG) load_wslice<D, PREC, CPW>(wreg, static_cast<const u32x4*>(net.wh), 0, wave, lane);

  // -- first layer: tanh(projection + W1x (x, y)), four columns per thread --
  {
    constexpr int RL = NTH / NG;   // rows in flight; thread: columns 4 n4 .. 4 n4 + 3
    const int rl = tid / NG;
    floatx4 wx, wy;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      wx[e] = kTwoLog2e * net.w1x[2 * (4 * n4 + e)];
      wy[e] = kTwoLog2e * net.w1x[2 * (4 * n4 + e) + 1];
    }
    for (int r = rl; r < R; r += RL) {
      const floatx4 ri = r_info[r];
      floatx4 c;
      if constexpr (SRC == SRC_GATHER) {
        c = *reinterpret_cast<const floatx4*>(&cs[__float_as_int(ri[2]) * D + 4 * n4]);
      } else {
        c = kTwoLog2e * *reinterpret_cast<const floatx4*>(A.C + r_bc[r] * D + 4 * n4);
      }
      float t[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) t[e] = ktanh_exp2(fmaf(ri[1], wy[e], fmaf(ri[0], wx[e], c[e])));
      store4<PREC>(&Hs[r * LDH + 4 * n4], t[0], t[1], t[2], t[3]);
    }
  }
  __syncthreads();

  // -- hidden layers on MFMA, output layer in the last epilogue -----------------
  hidden_and_output<D, R, PREC, CPW, WREG>(Hs, wreg, static_cast<const u32x4*>(net.wh), nb, po, lane, wave);

  // -- sum of the per-column-block partials (fixed order) and store -----------
  for (int r = tid; r < R; r += NTH) {
    const int64_t addr = r_addr[r];
    if (addr >= 0) {
      float s = 0.0f;
#pragma unroll
      for (int c = 0; c < NCOLB; ++c) s += po[c * R + r];
      const float val = s + net.b5[1];
      if constexpr (OUT == OUT_STORE) A.u_out[addr] = val;
      else if constexpr (OUT == OUT_ACCUM) A.u_out[addr] += val * r_info[r][3];
      else A.U[addr] = val;
    }
  }
}

// A tile shape: width, tile height, precision, output columns per wave and
// whether the hidden weights live in registers (else streamed from L2).
template <int D_, int R_, int PREC_, int CPW_, bool WREG_>
struct Shape {
  static constexpr int D = D_, R = R_, PREC = PREC_, CPW = CPW_;
  static constexpr bool WREG = WREG_, RS = false;
  static constexpr int NTH = (D / CPW) * 64;
  // waves per SIMD the register budget is sized for (HIP's second launch
  // bound): two 8-wave workgroups per CU, i.e. 128 VGPRs, where the LDS tile
  // allows it
  static constexpr int MINW = ((PREC != 0 && CPW == 32 && R <= 128) || (PREC == 0 && !WREG)) ? 2 * NTH / 256 : 1;
};

// ---------------------------------------------------------------------------
// Row-split bf16 tile. A 256-row tile is split by rows: each wave owns
// 32 PB consecutive rows (PB point blocks of 32) and computes all d units of
// every layer for them, so the activations never leave the registers: the
// converted accumulator of output block ob becomes the next layer's B operand
// for k groups 2 ob and 2 ob + 1 after one exchange between the half-waves
// (rs_operand), in the same k order as the column-split tile's, so both tiles
// give identical results. The hidden weights stream through LDS instead, half a
// layer at a time (64 KiB at d = 256) in two buffers: while the waves
// multiply with one half, the next half is copied into the other buffer by
// direct global-to-LDS loads, so one barrier per half layer is the only
// synchronisation. Each weight operand read from LDS serves PB MFMAs. The
// library launches PB = 1 (8 waves, two per SIMD); PB = 2 (4 waves, one per
// SIMD) needs more than the 256 architectural registers for its activations
// at d = 256 and ran slower.
// ---------------------------------------------------------------------------
// Next-layer B operand of one k group from eight tanh values of a lane's
// accumulator block: lane (point n, half h) holds units 4 h + 0..3 (v[0..3])
// and 8 + 4 h + 0..3 (v[4..7]) of the group's 16, the operand wants units
// 8 h + 0..7. One v_permlane32_swap per register pair moves the upper
// half-wave's first quarter and the lower half-wave's second quarter across.
template <int PREC>
__device__ __forceinline__ typename Mma<PREC>::T rs_operand(const float* v) {
  const uint32_t p0 = Mma<PREC>::pack(v[0], v[1]), p1 = Mma<PREC>::pack(v[2], v[3]);
  const uint32_t q0 = Mma<PREC>::pack(v[4], v[5]), q1 = Mma<PREC>::pack(v[6], v[7]);
  const auto s0 = __builtin_amdgcn_permlane32_swap(p0, q0, false, false);
  const auto s1 = __builtin_amdgcn_permlane32_swap(p1, q1, false, false);
  // s[0]: lower half-wave keeps its own, upper gets the lower's; s[1] the reverse
  return __builtin_bit_cast(typename Mma<PREC>::T, u32x4{s0[0], s1[0], s0[1], s1[1]});
}

template <int D_, int PB_, int PREC_ = 1, int R_ = 256>
struct RsShape {
  static constexpr int D = D_, R = R_, PREC = PREC_, CPW = 32, PB = PB_;
  static constexpr bool WREG = true, RS = true;
  static constexpr int NTH = 2 * R / PB, MINW = PB == 1 ? 2 : 1;
};

// R = 256: 8 waves, one workgroup per CU (143 KB of LDS at d = 256), the
// weights in half-layer steps. R = 128: 4 waves and quarter-layer steps
// (76 KB), so two workgroups share a CU and run out of step with each other:
// one's gather, projection, first layer and barrier waits overlap the
// other's MFMAs. Per row the arithmetic is the same in both.
template <int D, int TMODE, int OUT, int PB, int PREC = 1, int R = 256>
__device__ __forceinline__ void rs_body(const TileArgs& A, const int64_t row0) {
  typedef typename Mma<PREC>::T OT;   // 16-bit operand vector (bf16 or fp16)
  constexpr int NW = R / (32 * PB), NTH = 64 * NW;
  constexpr int T = n_targets<TMODE>();
  constexpr int NPMAX = (R - 1) / T + 2;
  constexpr int NOB = D / 32, NKG = D / 16;
  constexpr int NST = (R == 256 || D == 128) ? 2 : 4;   // weight steps per layer
  constexpr int HOB = NOB / NST;             // output blocks per step
  constexpr int HALF = HOB * NKG * 64;       // 16-byte pieces per step
  constexpr int PPT = HALF / NTH;            // pieces per thread
  static_assert(PPT * NTH == HALF && HOB * NST == NOB && NPMAX <= 8, "row-split tile");
  __shared__ __align__(16) u32x4 wbuf[2][HALF];
  __shared__ __align__(16) float gs[NPMAX * kNB];
  __shared__ __align__(16) float cs[NPMAX * D];
  __shared__ __align__(16) float nb[4 * D];    // k b2, k b3, k b4, -2 w5
  __shared__ __align__(16) float wxy[2 * D];   // k W1x[:, 0], k W1x[:, 1]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pn = lane & 31, hh = lane >> 5;
  const NetPtrs& net = A.net;
  const u32x4* whp = static_cast<const u32x4*>(net.wh);   // prepared bf16 weights, [ob][kg][lane][8]

  // step k (layer k / NST, output blocks HOB (k % NST) ..) into LDS buffer
  // `buf` with direct global-to-LDS loads (each lane's 16 bytes land at the
  // wave's base + 16 lane), so the copy holds no registers; completion is
  // awaited (vmcnt) before the barrier that publishes the buffer
  auto fetch = [&](int k, int buf) {
    int o = k * HALF;
    asm volatile("" : "+s"(o));
#pragma unroll
    for (int i = 0; i < PPT; ++i)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(whp + o + tid + i * NTH),
          (__attribute__((address_space(3))) void*)(&wbuf[buf][wave * 64 + i * NTH]), 16, 0, 0);
  };
  fetch(0, 0);

  for (int i = tid; i < 4 * D; i += NTH) nb[i] = i < 3 * D ? kTwoLog2e * net.bh[i] : -2.0f * net.w5[i - 3 * D];
  for (int i = tid; i < D; i += NTH) {
    wxy[i] = kTwoLog2e * net.w1x[2 * i];
    wxy[D + i] = kTwoLog2e * net.w1x[2 * i + 1];
  }

  // -- gather and bf16 boundary projection (once per placement) --------------
  const int64_t q0 = row0 / T;
  const int np = (int)((min(row0 + R, A.total_rows) - 1) / T - q0 + 1);
  for (int idx = tid; idx < np * kNB; idx += NTH) {
    const int sl = idx >> 7, k = idx & 127;
    int a, b, bi, bj;
    placement_of((int)(q0 + sl), A.colour, A.ux, a, b);
    boundary_local(k, bi, bj);
    gs[idx] = A.u_in[(int64_t)(kHalf * b + bj) * A.pitch + kHalf * a + bi];
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int cbk = wave; cbk < NOB; cbk += NW) {
    // A = the tile's boundary vectors (rows p < np), B = the 32-unit slice
    // cbk of W1g; registers 0..3 hold rows 4 hh .. 4 hh + 3 of unit col
    const int col = cbk * 32 + pn;
    const u32x4* wp = static_cast<const u32x4*>(net.w1gb) + (size_t)cbk * 8 * 64 + lane;
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll
    for (int kg = 0; kg < 8; ++kg) {
      u32x4 av = u32x4{0u, 0u, 0u, 0u};
      if (pn < np) {
        const floatx4 g0 = *reinterpret_cast<const floatx4*>(&gs[pn * kNB + 16 * kg + 8 * hh]);
        const floatx4 g1 = *reinterpret_cast<const floatx4*>(&gs[pn * kNB + 16 * kg + 8 * hh + 4]);
        av = u32x4{Mma<PREC>::pack(g0[0], g0[1]), Mma<PREC>::pack(g0[2], g0[3]), Mma<PREC>::pack(g1[0], g1[1]),
                   Mma<PREC>::pack(g1[2], g1[3])};
      }
      acc = Mma<PREC>::one(__builtin_bit_cast(OT, av), __builtin_bit_cast(OT, wp[kg * 64]), acc);
    }
    const float bb = net.b1[col];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * hh + v < np) cs[(4 * hh + v) * D + col] = kTwoLog2e * (acc[v] + bb);
  }

  // -- this lane's rows (one per point block) -----------------------------------
  bool valid[PB];
  int addr_i[PB], addr_j[PB], slot[PB];
  float x[PB], y[PB];
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int64_t row = row0 + (wave * PB + b) * 32 + pn;
    valid[b] = row < A.total_rows;
    const int64_t rr = valid[b] ? row : A.total_rows - 1;
    const int64_t q = rr / T;
    const int t = (int)(rr - q * T);
    int pa, pbb, ti, tj;
    placement_of((int)q, A.colour, A.ux, pa, pbb);
    target_local<TMODE>(t, ti, tj);
    x[b] = ti * (1.0f / kS);
    y[b] = tj * (1.0f / kS);
    slot[b] = (int)(q - q0);
    addr_i[b] = kHalf * pa + ti;
    addr_j[b] = kHalf * pbb + tj;
  }
  __syncthreads();   // projections, constants and the first half layer in LDS

  // -- first layer straight into B-operand registers (pairs packed by the
  // precision's converter) -------------------------------------------------
  OT H[2][PB][NKG];
#pragma unroll
  for (int kg = 0; kg < NKG; ++kg) {
    const int u0 = 16 * kg + 8 * hh;   // B operand: lane (point, half h) feeds units 16 kg + 8 h + 0..7
    u32x4 hb[PB];                      // the operand's four registers, two units each
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const floatx4 wx = *reinterpret_cast<const floatx4*>(&wxy[u0 + 4 * g]);
      const floatx4 wy = *reinterpret_cast<const floatx4*>(&wxy[D + u0 + 4 * g]);
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        const floatx4 c = *reinterpret_cast<const floatx4*>(&cs[slot[b] * D + u0 + 4 * g]);
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = ktanh_exp2(fmaf(y[b], wy[e], fmaf(x[b], wx[e], c[e])));
        hb[b][2 * g] = Mma<PREC>::pack(v[0], v[1]);
        hb[b][2 * g + 1] = Mma<PREC>::pack(v[2], v[3]);
      }
    }
#pragma unroll
    for (int b = 0; b < PB; ++b) H[0][b][kg] = __builtin_bit_cast(OT, hb[b]);
  }

  // -- hidden layers: 3 NST weight steps --------------------------------------
  float s[PB];
#pragma unroll
  for (int b = 0; b < PB; ++b) s[b] = 0.0f;
#pragma unroll
  for (int k = 0; k < 3 * NST; ++k) {
    const int l = k / NST, hf = k % NST;
    OT(&hin)[PB][NKG] = H[l & 1];
    OT(&hout)[PB][NKG] = H[(l + 1) & 1];
    // the other buffer's step was finished by every wave before the last barrier
    if (k < 3 * NST - 1) fetch(k + 1, (k + 1) & 1);
    const u32x4* wb = wbuf[k & 1] + lane;
    // weight operand i of the step (output block i / NKG, k group
    // i % NKG) comes from a ring filled four operands ahead and feeds PB
    // MFMAs; the tanh (or output dot) of the previous output block's 16 PB
    // accumulator elements is spread over the block's MFMAs so both pipes
    // stay busy
    constexpr int NI = HOB * NKG, RING = 4, EPK = 16 / NKG;   // epilogue elements per k group and block
    OT ar[RING];
#pragma unroll
    for (int i = 0; i < RING; ++i) ar[i] = __builtin_bit_cast(OT, wb[i * 64]);
    floatx16 acc[2][PB];
    float ev[PB][16];
    float dsum[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) dsum[b] = 0.0f;
#pragma unroll
    for (int j = 0; j <= HOB; ++j) {
      const int obp = hf * HOB + j - 1;   // block whose epilogue runs now
      if (j < HOB) {
        const floatx16 bias = bias_acc(nb + l * D + 32 * (hf * HOB + j) + 4 * hh);
#pragma unroll
        for (int b = 0; b < PB; ++b) acc[j & 1][b] = bias;
      }
      floatx4 w5v[4];
      if (l == 2 && j > 0) {
#pragma unroll
        for (int g = 0; g < 4; ++g) w5v[g] = *reinterpret_cast<const floatx4*>(nb + 3 * D + 32 * obp + 4 * hh + 8 * g);
      }
#pragma unroll
      for (int kg = 0; kg < NKG; ++kg) {
        const int i = j * NKG + kg;
        if (j < HOB) {
#pragma unroll
          for (int b = 0; b < PB; ++b) acc[j & 1][b] = Mma<PREC>::one(ar[i % RING], hin[b][kg], acc[j & 1][b]);
          if (i + RING < NI) ar[i % RING] = __builtin_bit_cast(OT, wb[(i + RING) * 64]);
        }
        if (j > 0) {
#pragma unroll
          for (int b = 0; b < PB; ++b)
#pragma unroll
            for (int ee = 0; ee < EPK; ++ee) {
              const int e = kg * EPK + ee;   // accumulator element 0..15
              const float c = acc[(j - 1) & 1][b][e];
              if (l < 2) {
                ev[b][e] = ktanh_exp2(c);
                if ((e & 7) == 7) {
                  const int h2 = e >> 3;
                  hout[b][2 * obp + h2] = rs_operand<PREC>(ev[b] + 8 * h2);
                }
              } else {
                dsum[b] = fmaf(w5v[e >> 2][e & 3], rsig_exp2(c), dsum[b]);
                if (e == 15) {
                  dsum[b] += __shfl_xor(dsum[b], 32);
                  s[b] += dsum[b];
                  dsum[b] = 0.0f;
                }
              }
            }
        }
      }
    }
    if (k < 3 * NST - 1) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }

  // -- output ----------------------------------------------------------------
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    if (valid[b] && hh == 0) {
      const int64_t addr = (int64_t)addr_j[b] * A.pitch + addr_i[b];
      const float val = s[b] + net.b5[1];
      if constexpr (OUT == OUT_STORE) A.u_out[addr] = val;
      else A.u_out[addr] += val * (cover_inv(addr_i[b], kS * A.ux) * cover_inv(addr_j[b], kS * A.uy));
    }
  }
}

template <class S, int TMODE, int SRC, int OUT>
__global__ __launch_bounds__(S::NTH, S::MINW) void tile_kernel(TileArgs A) {
  if constexpr (S::RS) {
    if constexpr (SRC == SRC_GATHER && OUT != OUT_LINEAR)
      rs_body<S::D, TMODE, OUT, S::PB, S::PREC, S::R>(A, (A.block0 + blockIdx.x) * S::R);
  } else {
    tile_body<S::D, S::R, TMODE, S::PREC, SRC, OUT, S::CPW, S::WREG>(A, (A.block0 + blockIdx.x) * S::R);
  }
}

// Batched independent domains in one persistent launch per colour: block b
// takes tiles b, b + gridDim.x, ...; tile t belongs to the domain d with
// tile_begin[d] <= t < tile_begin[d + 1] and covers rows
// [(t - tile_begin[d]) R, ... + R) of that domain's phase.
// Tiles per launch: keeps the work-items of one launch below 2^32.
constexpr int64_t kMaxTilesPerLaunch = 1 << 22;

struct MultiArgs {
  TileArgs base;             // network; colour
  const float* field_in;     // packed fields (domain offsets are relative to these)
  float* field_out;
  const DomEntry* doms;      // [n_domains]
  const int32_t* tile_begin; // [n_domains + 1] for this colour and target set
  int n_domains;
  int64_t n_tiles;
  int64_t tile0;             // row-split tile: first tile of this launch
  int64_t n_launch;          // row-split tile: tiles of this launch
};

// The row-split tile runs one tile per workgroup by default (its registers
// are full); with PERSIST a grid of one workgroup per CU walks the launch's
// tiles, the network pointers made opaque per tile so that no tile-invariant
// load is hoisted across tiles (which spilled). The other shapes always take
// tiles round-robin in a persistent grid.
template <class S, int TMODE, int OUT, bool PERSIST = false>
__global__ __launch_bounds__(S::NTH, S::MINW) void tile_kernel_multi(MultiArgs M) {
  constexpr int T = n_targets<TMODE>();
  const int ca = M.base.colour & 1, cb = M.base.colour >> 1;
  auto run_tile = [&](int64_t t) {
    int lo = 0, hi = M.n_domains - 1;       // last d with tile_begin[d] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (M.tile_begin[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const DomEntry e = M.doms[lo];
    TileArgs A = M.base;
    if constexpr (PERSIST) {
      int z = 0;
      asm volatile("" : "+s"(z));
      A.net.w1gT += z;
      A.net.w1gb = static_cast<const u32x4*>(A.net.w1gb) + z;
      A.net.w1x += z;
      A.net.b1 += z;
      A.net.bh += z;
      A.net.w5 += z;
      A.net.b5 += z;
      A.net.wh = static_cast<const u32x4*>(A.net.wh) + z;
    }
    A.u_in = M.field_in + e.offset;
    A.u_out = M.field_out + e.offset;
    A.pitch = e.pitch;
    A.ux = e.ux;
    A.uy = e.uy;
    A.total_rows = (int64_t)(e.ux - ca) * (e.uy - cb) * T;
    if constexpr (S::RS) rs_body<S::D, TMODE, OUT, S::PB, S::PREC, S::R>(A, (t - M.tile_begin[lo]) * S::R);
    else tile_body<S::D, S::R, TMODE, S::PREC, SRC_GATHER, OUT, S::CPW, S::WREG>(A, (t - M.tile_begin[lo]) * S::R);
  };
  if constexpr (S::RS && !PERSIST) {
    run_tile(M.tile0 + blockIdx.x);
  } else if constexpr (S::RS) {
    const int64_t end = M.tile0 + M.n_launch;
    for (int64_t t = M.tile0 + blockIdx.x; t < end; t += gridDim.x) {
      run_tile(t);
      __syncthreads();   // the next tile reuses the LDS
    }
  } else {
    for (int64_t t = blockIdx.x; t < M.n_tiles; t += gridDim.x) {
      run_tile(t);
      __syncthreads();   // the next tile reuses the LDS
    }
  }
}

// Tile shapes by (width, precision, tile code): fp32 32 (streamed weights),
// 64 (register weights), 64 | MF_TILE_STREAM (streamed); bf16 64, 128, 256,
// 128 or 256 | MF_TILE_WIDE (64 columns per wave) and 128 or 256 |
// MF_TILE_ROWSPLIT (row-split tiles); fp16 the bf16 codes without
// MF_TILE_WIDE. The caller has validated the code.
template <int D, class F>
static hipError_t with_shape_d(int prec, int code, F&& f) {
  const int r = code & 0xffff;
  if (prec == MF_BF16) {
    if (code & MF_TILE_ROWSPLIT) return r == 128 ? f(RsShape<D, 1, 1, 128>{}) : f(RsShape<D, 1>{});
    if (code & MF_TILE_WIDE) return r == 256 ? f(Shape<D, 256, 1, 64, true>{}) : f(Shape<D, 128, 1, 64, true>{});
    if (r == 256) return f(Shape<D, 256, 1, 32, true>{});
    if (r == 128) return f(Shape<D, 128, 1, 32, true>{});
    return f(Shape<D, 64, 1, 32, true>{});
  }
  if (prec == MF_FP16) {   // the same tiles on fp16 operands (no 64-column forms)
    if (code & MF_TILE_ROWSPLIT) return r == 128 ? f(RsShape<D, 1, 2, 128>{}) : f(RsShape<D, 1, 2>{});
    if (r == 256) return f(Shape<D, 256, 2, 32, true>{});
    if (r == 128) return f(Shape<D, 128, 2, 32, true>{});
    return f(Shape<D, 64, 2, 32, true>{});
  }
  if (r == 64) return (code & MF_TILE_STREAM) ? f(Shape<D, 64, 0, 32, false>{}) : f(Shape<D, 64, 0, 32, true>{});
  return f(Shape<D, 32, 0, 32, false>{});
}

template <class F>
static hipError_t with_shape(int width, int prec, int code, F&& f) {
  return width == 256 ? with_shape_d<256>(prec, code, f) : with_shape_d<128>(prec, code, f);
}

template <class S, int TMODE, int OUT>
static hipError_t launch_multi(MultiArgs m, int n_cu, bool persist, hipStream_t s) {
  if (m.n_tiles == 0) return hipSuccess;
  if constexpr (S::RS) {
    for (int64_t t0 = 0; t0 < m.n_tiles; t0 += kMaxTilesPerLaunch) {
      m.tile0 = t0;
      const int64_t n = std::min<int64_t>(m.n_tiles - t0, kMaxTilesPerLaunch);
      m.n_launch = n;
      if (persist) {
        static int per_cu_p = 0;
        if (per_cu_p == 0) {
          int nb = 0;
          if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tile_kernel_multi<S, TMODE, OUT, true>, S::NTH, 0) !=
                  hipSuccess ||
              nb < 1)
            nb = 1;
          per_cu_p = nb;
        }
        const int64_t grid = std::min<int64_t>(n, (int64_t)per_cu_p * n_cu);
        hipLaunchKernelGGL((tile_kernel_multi<S, TMODE, OUT, true>), dim3((unsigned)grid), dim3(S::NTH), 0, s, m);
      } else {
        hipLaunchKernelGGL((tile_kernel_multi<S, TMODE, OUT>), dim3((unsigned)n), dim3(S::NTH), 0, s, m);
      }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tile_kernel_multi<S, TMODE, OUT>, S::NTH, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    per_cu = nb;
  }
  const int64_t grid = std::min<int64_t>(m.n_tiles, (int64_t)per_cu * n_cu);
  hipLaunchKernelGGL((tile_kernel_multi<S, TMODE, OUT>), dim3((unsigned)grid), dim3(S::NTH), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_phase_multi(const NetPtrs& net, int width, int prec, int targets, bool accumulate,
                              int tile_rows, const float* field_in, float* field_out,
                              const DomEntry* doms, const int32_t* tile_begin, int n_domains,
                              int64_t n_tiles, int colour, int n_cu, hipStream_t s) {
  MultiArgs m{};
  m.base.net = net;
  m.base.colour = colour;
  m.field_in = field_in;
  m.field_out = field_out;
  m.doms = doms;
  m.tile_begin = tile_begin;
  m.n_domains = n_domains;
  m.n_tiles = n_tiles;
  const bool persist = (tile_rows & MF_TILE_PERSIST) != 0;
  return with_shape(width, prec, tile_rows, [&](auto sh) {
    typedef decltype(sh) S;
    if (accumulate)
      return targets == MF_CROSS ? launch_multi<S, 0, OUT_ACCUM>(m, n_cu, persist, s)
                                 : launch_multi<S, 1, OUT_ACCUM>(m, n_cu, persist, s);
    return targets == MF_CROSS ? launch_multi<S, 0, OUT_STORE>(m, n_cu, persist, s)
                               : launch_multi<S, 1, OUT_STORE>(m, n_cu, persist, s);
  });
}

template <class S, int TMODE, int SRC, int OUT>
static hipError_t launch_tile(TileArgs a, hipStream_t s) {
  const int64_t blocks = (a.total_rows + S::R - 1) / S::R;
  for (int64_t b0 = 0; b0 < blocks; b0 += kMaxTilesPerLaunch) {
    a.block0 = b0;
    const int64_t n = std::min<int64_t>(blocks - b0, kMaxTilesPerLaunch);
    hipLaunchKernelGGL((tile_kernel<S, TMODE, SRC, OUT>), dim3((unsigned)n), dim3(S::NTH), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static int64_t colour_count(int ux, int uy, int colour) {
  return (int64_t)(ux - (colour & 1)) * (uy - (colour >> 1));
}

hipError_t launch_phase(const NetPtrs& net, int width, int prec, int targets, bool accumulate,
                        int tile_rows, const PhaseArgs& p, hipStream_t s) {
  TileArgs a{};
  a.net = net;
  a.u_in = p.u_in;
  a.u_out = p.u_out;
  a.pitch = p.pitch;
  a.ux = p.ux;
  a.uy = p.uy;
  a.colour = p.colour;
  const int T = targets == MF_INTERIOR ? kInterior : kCross;
  a.total_rows = colour_count(p.ux, p.uy, p.colour) * T;
  if (a.total_rows == 0) return hipSuccess;
  return with_shape(width, prec, tile_rows, [&](auto sh) {
    typedef decltype(sh) S;
    if (accumulate)
      return targets == MF_CROSS ? launch_tile<S, 0, SRC_GATHER, OUT_ACCUM>(a, s)
                                 : launch_tile<S, 1, SRC_GATHER, OUT_ACCUM>(a, s);
    return targets == MF_CROSS ? launch_tile<S, 0, SRC_GATHER, OUT_STORE>(a, s)
                               : launch_tile<S, 1, SRC_GATHER, OUT_STORE>(a, s);
  });
}

// ---------------------------------------------------------------------------
// sdnet_forward: projection per boundary condition, then the same tile
// kernel over (condition, point) rows.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(D) void projection_kernel(NetPtrs net, const float* __restrict__ G,
                                                       int64_t n_bc, float* __restrict__ C) {
  constexpr int NBC = 8;
  __shared__ float gsh[NBC * kNB];
  const int64_t bc0 = (int64_t)blockIdx.x * NBC;
  for (int idx = threadIdx.x; idx < NBC * kNB; idx += D) {
    const int b = idx >> 7, k = idx & 127;
    gsh[idx] = (bc0 + b < n_bc) ? G[(bc0 + b) * kNB + k] : 0.0f;
  }
  __syncthreads();
  const int n = threadIdx.x;
  float acc[NBC];
#pragma unroll
  for (int b = 0; b < NBC; ++b) acc[b] = net.b1[n];
#pragma unroll 8
  for (int k = 0; k < kNB; ++k) {
    const float w = net.w1gT[k * D + n];
#pragma unroll
    for (int b = 0; b < NBC; ++b) acc[b] = fmaf(w, gsh[b * kNB + k], acc[b]);
  }
#pragma unroll
  for (int b = 0; b < NBC; ++b)
    if (bc0 + b < n_bc) C[(bc0 + b) * D + n] = acc[b];
}

hipError_t launch_projection(const NetPtrs& net, int width, const float* G, int64_t n_bc,
                             float* C, hipStream_t s) {
  const int64_t blocks = (n_bc + 7) / 8;
  if (blocks == 0) return hipSuccess;
  if (width == 256)
    hipLaunchKernelGGL(projection_kernel<256>, dim3((unsigned)blocks), dim3(256), 0, s, net, G, n_bc, C);
  else
    hipLaunchKernelGGL(projection_kernel<128>, dim3((unsigned)blocks), dim3(128), 0, s, net, G, n_bc, C);
  return hipGetLastError();
}

hipError_t launch_forward_rows(const NetPtrs& net, int width, int prec, const float* C,
                               const float* X, int64_t n_bc, int64_t n_pts, int x_per_bc,
                               float* U, hipStream_t s) {
  TileArgs a{};
  a.net = net;
  a.C = C;
  a.X = X;
  a.n_pts = n_pts;
  a.x_per_bc = x_per_bc;
  a.U = U;
  a.total_rows = n_bc * n_pts;
  if (a.total_rows == 0) return hipSuccess;
  return with_shape(width, prec, 64, [&](auto sh) { return launch_tile<decltype(sh), 0, SRC_C, OUT_LINEAR>(a, s); });
}

// ---------------------------------------------------------------------------
// Assembly initialisation: ring copied from u, interior zeroed (the four
// colour phases then accumulate prediction / cover count).
// ---------------------------------------------------------------------------
__global__ void assembly_init_kernel(const float* __restrict__ u, float* __restrict__ u_out,
                                     int64_t pitch, int nx, int ny) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / nx), i = (int)(idx - (int64_t)j * nx);
    const int64_t o = (int64_t)j * pitch + i;
    const bool ring = i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
    u_out[o] = ring ? u[o] : 0.0f;
  }
}

hipError_t launch_assembly_init(const float* u, float* u_out, int64_t pitch, int ux, int uy,
                                hipStream_t s) {
  const int nx = kS * ux + 1, ny = kS * uy + 1;
  const int64_t n = (int64_t)nx * ny;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(assembly_init_kernel, dim3(blocks), dim3(256), 0, s, u, u_out, pitch, nx, ny);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Additive (parallel Schwarz) sweep: every placement reads the old field u and
// the targets of the new field take the mean of the predictions covering
// them. A target point is covered 1 / (cover_inv(i) cover_inv(j)) times for
// either target set, so the colour phases accumulate pred * cover_inv^2 into
// un, which starts as u with its target points zeroed; then the targets are
// copied back into u.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool is_target_point(int i, int j, int nx, int ny, int interior) {
  const bool inner = i > 0 && j > 0 && i < nx - 1 && j < ny - 1;
  return inner && (interior || (i & 15) == 0 || (j & 15) == 0);
}

__global__ void additive_init_kernel(const float* __restrict__ u, float* __restrict__ un, int64_t pitch,
                                     int nx, int ny, int interior) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / nx), i = (int)(idx - (int64_t)j * nx);
    const int64_t o = (int64_t)j * pitch + i;
    un[o] = is_target_point(i, j, nx, ny, interior) ? 0.0f : u[o];
  }
}

__global__ void additive_copy_kernel(const float* __restrict__ un, float* __restrict__ u, int64_t pitch,
                                     int nx, int ny, int interior) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / nx), i = (int)(idx - (int64_t)j * nx);
    if (is_target_point(i, j, nx, ny, interior)) {
      const int64_t o = (int64_t)j * pitch + i;
      u[o] = un[o];
    }
  }
}

hipError_t launch_additive_init(const float* u, float* un, int64_t pitch, int ux, int uy, int targets,
                                hipStream_t s) {
  const int nx = kS * ux + 1, ny = kS * uy + 1;
  const int blocks = (int)std::min<int64_t>(((int64_t)nx * ny + 255) / 256, 4096);
  hipLaunchKernelGGL(additive_init_kernel, dim3(blocks), dim3(256), 0, s, u, un, pitch, nx, ny,
                     targets == MF_INTERIOR ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_additive_copy(const float* un, float* u, int64_t pitch, int ux, int uy, int targets,
                                hipStream_t s) {
  const int nx = kS * ux + 1, ny = kS * uy + 1;
  const int blocks = (int)std::min<int64_t>(((int64_t)nx * ny + 255) / 256, 4096);
  hipLaunchKernelGGL(additive_copy_kernel, dim3(blocks), dim3(256), 0, s, un, u, pitch, nx, ny,
                     targets == MF_INTERIOR ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Delta test (Alg. 2): relative L2 change of the skeleton values. The
// skeleton is stored compactly: the 2 uy + 1 full stride rows first, then
// the 2 ux + 1 stride columns without the points already on stride rows.
// ---------------------------------------------------------------------------
int64_t skeleton_count(int ux, int uy) {
  return (int64_t)(2 * uy + 1) * (kS * ux + 1) + (int64_t)(2 * ux + 1) * (30 * uy);
}

__device__ __forceinline__ void skeleton_point(int64_t s, int ux, int uy, int& i, int& j) {
  const int nx = kS * ux + 1;
  const int64_t nrow = (int64_t)(2 * uy + 1) * nx;
  if (s < nrow) {
    const int r = (int)(s / nx);
    i = (int)(s - (int64_t)r * nx);
    j = kHalf * r;
  } else {
    const int64_t s2 = s - nrow;
    const int per = 30 * uy;
    const int c = (int)(s2 / per);
    const int m = (int)(s2 - (int64_t)c * per);
    const int seg = m / 15, off = m - seg * 15;
    j = kHalf * seg + off + 1;
    i = kHalf * c;
  }
}

__global__ void skeleton_snapshot_kernel(const float* __restrict__ u, int64_t pitch, int ux,
                                         int uy, float* __restrict__ skel) {
  const int64_t n = (2 * (int64_t)uy + 1) * (kS * ux + 1) + (2 * (int64_t)ux + 1) * (30 * uy);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    skeleton_point(s, ux, uy, i, j);
    skel[s] = u[(int64_t)j * pitch + i];
  }
}

__device__ __forceinline__ float block_sum_256(float v, float* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  float t = 0.0f;
  if (threadIdx.x == 0) t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void delta_partial_kernel(const float* __restrict__ u, int64_t pitch,
                                                            int ux, int uy,
                                                            const float* __restrict__ skel,
                                                            float* __restrict__ part) {
  __shared__ float sh[4];
  const int64_t n = (2 * (int64_t)uy + 1) * (kS * ux + 1) + (2 * (int64_t)ux + 1) * (30 * uy);
  float num = 0.0f, den = 0.0f;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    skeleton_point(s, ux, uy, i, j);
    const float old = skel[s];
    const float dv = u[(int64_t)j * pitch + i] - old;
    num = fmaf(dv, dv, num);
    den = fmaf(old, old, den);
  }
  const float tn = block_sum_256(num, sh);
  const float td = block_sum_256(den, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = tn;
    part[kDeltaBlocks + blockIdx.x] = td;
  }
}

__global__ __launch_bounds__(256) void delta_final_kernel(const float* __restrict__ part, int nb,
                                                          float* __restrict__ dres) {
  __shared__ float sh[4];
  float num = 0.0f, den = 0.0f;
  for (int b = threadIdx.x; b < nb; b += 256) {
    num += part[b];
    den += part[kDeltaBlocks + b];
  }
  const float tn = block_sum_256(num, sh);
  const float td = block_sum_256(den, sh);
  if (threadIdx.x == 0) {
    dres[0] = tn;
    dres[1] = td;
  }
}

hipError_t launch_skeleton_snapshot(const float* u, int64_t pitch, int ux, int uy, float* skel,
                                    hipStream_t s) {
  const int64_t n = skeleton_count(ux, uy);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(skeleton_snapshot_kernel, dim3(blocks), dim3(256), 0, s, u, pitch, ux, uy, skel);
  return hipGetLastError();
}

hipError_t launch_delta(const float* u, int64_t pitch, int ux, int uy, const float* skel,
                        float* part, float* dres, hipStream_t s) {
  const int64_t n = skeleton_count(ux, uy);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, kDeltaBlocks);
  hipLaunchKernelGGL(delta_partial_kernel, dim3(blocks), dim3(256), 0, s, u, pitch, ux, uy, skel, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(delta_final_kernel, dim3(1), dim3(256), 0, s, part, blocks, dres);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Check mode: subdomain solver = linear operator Hop [T x 128].
// ---------------------------------------------------------------------------
template <int TMODE, int OUT>
__global__ __launch_bounds__(256) void operator_kernel(const float* __restrict__ Hop, PhaseArgs p, int q0) {
  constexpr int T = n_targets<TMODE>();
  __shared__ float g[kNB];
  int a, b;
  placement_of(q0 + (int)blockIdx.x, p.colour, p.ux, a, b);
  if (threadIdx.x < kNB) {
    int bi, bj;
    boundary_local(threadIdx.x, bi, bj);
    g[threadIdx.x] = p.u_in[(int64_t)(kHalf * b + bj) * p.pitch + kHalf * a + bi];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += 256) {
    const float* h = Hop + (int64_t)t * kNB;
    float s = 0.0f;
    for (int k = 0; k < kNB; ++k) s = fmaf(h[k], g[k], s);
    int ti, tj;
    target_local<TMODE>(t, ti, tj);
    const int gi = kHalf * a + ti, gj = kHalf * b + tj;
    const int64_t o = (int64_t)gj * p.pitch + gi;
    if constexpr (OUT == OUT_STORE) p.u_out[o] = s;
    else p.u_out[o] += s * cover_inv(gi, kS * p.ux) * cover_inv(gj, kS * p.uy);
  }
}

hipError_t launch_operator_phase(const float* Hop, int targets, bool accumulate,
                                 const PhaseArgs& p, hipStream_t s) {
  const int64_t n = colour_count(p.ux, p.uy, p.colour);
  for (int64_t q0 = 0; q0 < n; q0 += kMaxTilesPerLaunch) {
    const dim3 grid((unsigned)std::min<int64_t>(n - q0, kMaxTilesPerLaunch));
    if (accumulate)
      hipLaunchKernelGGL((operator_kernel<1, OUT_ACCUM>), grid, dim3(256), 0, s, Hop, p, (int)q0);
    else if (targets == MF_CROSS)
      hipLaunchKernelGGL((operator_kernel<0, OUT_STORE>), grid, dim3(256), 0, s, Hop, p, (int)q0);
    else
      hipLaunchKernelGGL((operator_kernel<1, OUT_STORE>), grid, dim3(256), 0, s, Hop, p, (int)q0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mf

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
__global__ void prepare_net_kernel(const float* __restrict__ params, int d, int prec,
                                   float* __restrict__ w1gT, float* __restrict__ w1x,
                                   float* __restrict__ b1, void* __restrict__ wh,
                                   float* __restrict__ bh, float* __restrict__ w5,
                                   float* __restrict__ b5) {
  const int64_t off_b1 = (int64_t)d * 130;
  const int64_t off_w2 = off_b1 + d;
  const int64_t lstride = (int64_t)d * d + d;
  const int64_t off_w5 = off_w2 + 3 * lstride;
  const int64_t off_b5 = off_w5 + d;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;

  for (int64_t idx = tid; idx < 128 * (int64_t)d; idx += nthr) {
    const int64_t k = idx / d, n = idx - k * d;
    w1gT[idx] = params[n * 130 + k];
  }
  for (int64_t n = tid; n < d; n += nthr) {
    w1x[2 * n] = params[n * 130 + 128];
    w1x[2 * n + 1] = params[n * 130 + 129];
    b1[n] = params[off_b1 + n];
    w5[n] = params[off_w5 + n];
    for (int l = 0; l < 3; ++l) bh[l * d + n] = params[off_w2 + l * lstride + (int64_t)d * d + n];
  }
  if (tid == 0) b5[0] = params[off_b5];

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
      static_cast<uint16_t*>(wh)[idx] = bf16_bits(params[off_w2 + l * lstride + (int64_t)j * d + k]);
    }
  }
}

hipError_t launch_prepare_net(const float* params, int width, int prec, const NetLayout& L,
                              void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  hipLaunchKernelGGL(prepare_net_kernel, dim3(256), dim3(256), 0, s, params, width, prec,
                     reinterpret_cast<float*>(base + L.w1gT), reinterpret_cast<float*>(base + L.w1x),
                     reinterpret_cast<float*>(base + L.b1), static_cast<void*>(base + L.wh),
                     reinterpret_cast<float*>(base + L.bh), reinterpret_cast<float*>(base + L.w5),
                     reinterpret_cast<float*>(base + L.b5));
  return hipGetLastError();
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
};

template <int PREC> struct HType { typedef float T; };
template <> struct HType<1> { typedef uint16_t T; };

template <int PREC>
__device__ __forceinline__ void h_store(typename HType<PREC>::T* p, float v) {
  if constexpr (PREC == 0) *p = v; else *p = bf16_bits(v);
}
template <int PREC>
__device__ __forceinline__ float h_load(const typename HType<PREC>::T* p) {
  if constexpr (PREC == 0) return *p; else return bf16_to_f32(*p);
}

// Three hidden layers with bf16 operands and float32 accumulation. Each wave
// owns 32 output columns and keeps its slice of the layer's weights in
// registers (D/16 bf16x8 operands); it walks the tile's 32-row blocks with
// one barrier per block, so the tanh epilogue of block rb-1 (written back
// in place: every wave has finished reading those rows once it passed the
// previous barrier) overlaps the MFMAs of block rb.
template <int D, int R, int CPW>
__device__ __forceinline__ void hidden_layers_bf16(uint16_t* Hs, const u32x4* wh, const float* bh,
                                                   int lane, int wave) {
  constexpr int RB = R / 32, KG = D / 16, LDH = D + 8, NCB = CPW / 32;
  const int arow = lane & 31, ahalf = lane >> 5;
#pragma unroll 1
  for (int l = 0; l < 3; ++l) {
    bf16x8 breg[NCB][KG];
    float bj[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const u32x4* wsw = wh + (size_t)l * (D * D / 8) + (size_t)(wave * NCB + cb) * KG * 64 + lane;
#pragma unroll
      for (int kg = 0; kg < KG; ++kg) breg[cb][kg] = __builtin_bit_cast(bf16x8, wsw[kg * 64]);
      bj[cb] = bh[l * D + (wave * NCB + cb) * 32 + arow];
    }
    floatx16 prev[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) prev[cb][v] = 0.0f;
#pragma unroll 1
    for (int rb = 0; rb <= RB; ++rb) {
      floatx16 acc[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[cb][v] = 0.0f;
      if (rb < RB) {
        const uint16_t* ap = Hs + (rb * 32 + arow) * LDH + 8 * ahalf;
#pragma unroll
        for (int kg = 0; kg < KG; ++kg) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(ap + kg * 16));
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma32x32x16_bf16(av, breg[cb][kg], acc[cb]);
        }
      }
      if (rb > 0) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          uint16_t* op = Hs + ((rb - 1) * 32) * LDH + (wave * NCB + cb) * 32 + arow;
#pragma unroll
          for (int v = 0; v < 16; v += 2) {
            uint16_t h0, h1;
            bf16_pair(tanh_fast(prev[cb][v] + bj[cb]), tanh_fast(prev[cb][v + 1] + bj[cb]), h0, h1);
            op[acc_row(lane, v) * LDH] = h0;
            op[acc_row(lane, v + 1) * LDH] = h1;
          }
        }
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) prev[cb] = acc[cb];
      __syncthreads();
    }
  }
}

// The same pipeline with float32 operands: each wave holds its 32-column
// weight slice as D/8 float4 MFMA operands (128 VGPRs at d = 256) for the
// whole layer, so the k loop issues LDS reads and MFMAs only.
template <int D, int R>
__device__ __forceinline__ void hidden_layers_f32(float* Hs, const floatx4* wh, const float* bh, int lane,
                                                  int wave) {
  constexpr int RB = R / 32, KG = D / 8, LDH = D + 4;
  const int arow = lane & 31, ahalf = lane >> 5;
  const int j = wave * 32 + arow;
#pragma unroll 1
  for (int l = 0; l < 3; ++l) {
    floatx4 breg[KG];
    const floatx4* wsw = wh + (size_t)l * (D * D / 4) + (size_t)wave * KG * 64 + lane;
#pragma unroll
    for (int kg = 0; kg < KG; ++kg) breg[kg] = wsw[kg * 64];
    const float bj = bh[l * D + j];
    floatx16 prev;
#pragma unroll
    for (int v = 0; v < 16; ++v) prev[v] = 0.0f;
#pragma unroll 1
    for (int rb = 0; rb <= RB; ++rb) {
      floatx16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
      if (rb < RB) {
        const float* ap = Hs + (rb * 32 + arow) * LDH + 4 * ahalf;
#pragma unroll
        for (int kg = 0; kg < KG; ++kg) {
          const floatx4 av = *reinterpret_cast<const floatx4*>(ap + kg * 8);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc = mfma32x32x2(av[e], breg[kg][e], acc);
        }
      }
      if (rb > 0) {
        float* op = Hs + ((rb - 1) * 32) * LDH + j;
#pragma unroll
        for (int v = 0; v < 16; ++v) op[acc_row(lane, v) * LDH] = tanh_fast(prev[v] + bj);
      }
      prev = acc;
      __syncthreads();
    }
  }
}

template <int D, int R, int TMODE, int PREC, int SRC, int OUT, int CPW = 32>
__device__ __forceinline__ void tile_body(const TileArgs& A, const int64_t row0) {
  static_assert(CPW == 32 || (CPW == 64 && PREC == 1), "64 columns per wave: bf16 only");
  constexpr int NTH = (D / CPW) * 64;        // one wave per CPW output columns
  constexpr int RB = R / 32;                 // 32-row MFMA blocks per tile
  constexpr int T = n_targets<TMODE>();
  constexpr int NPMAX = SRC == SRC_GATHER ? (R - 1) / T + 2 : 1;
  constexpr int LDH = PREC == 0 ? D + 4 : D + 8;   // padded row (elements)
  typedef typename HType<PREC>::T HT;

  __shared__ __align__(16) HT Hs[R * LDH];
  __shared__ float gs[NPMAX * kNB];
  __shared__ float cs[NPMAX * D];
  __shared__ int r_slot[R];
  __shared__ float r_x[R], r_y[R], r_w[R];
  __shared__ int64_t r_addr[R];
  __shared__ int64_t r_bc[SRC == SRC_C ? R : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const NetPtrs& net = A.net;

  // -- rows of this tile -----------------------------------------------------
  int64_t q0 = 0;
  int np = 0;
  if constexpr (SRC == SRC_GATHER) {
    const int64_t last = min(row0 + R, A.total_rows) - 1;
    q0 = row0 / T;
    np = (int)(last / T - q0 + 1);
  }
  for (int rt = tid; rt < R; rt += NTH) {
    const int tid = rt;
    const int64_t row = row0 + tid;
    const bool valid = row < A.total_rows;
    const int64_t rr = valid ? row : A.total_rows - 1;
    if constexpr (SRC == SRC_GATHER) {
      const int q = (int)(rr / T), t = (int)(rr - (int64_t)q * T);
      int a, b, ti, tj;
      placement_of(q, A.colour, A.ux, a, b);
      target_local<TMODE>(t, ti, tj);
      const int gi = kHalf * a + ti, gj = kHalf * b + tj;
      r_slot[tid] = (int)(q - q0);
      r_x[tid] = ti * (1.0f / kS);
      r_y[tid] = tj * (1.0f / kS);
      r_w[tid] = cover_inv(gi, kS * A.ux) * cover_inv(gj, kS * A.uy);
      r_addr[tid] = valid ? (int64_t)gj * A.pitch + gi : -1;
    } else {
      const int64_t bc = rr / A.n_pts, pt = rr - bc * A.n_pts;
      const float* xp = A.x_per_bc ? A.X + 2 * rr : A.X + 2 * pt;
      r_x[tid] = xp[0];
      r_y[tid] = xp[1];
      r_bc[tid] = bc;
      r_addr[tid] = valid ? rr : -1;
    }
  }

  // -- gather + boundary projection (once per placement) --------------------
  if constexpr (SRC == SRC_GATHER) {
    for (int idx = tid; idx < np * kNB; idx += NTH) {
      const int s = idx >> 7, k = idx & 127;
      int a, b, bi, bj;
      placement_of((int)(q0 + s), A.colour, A.ux, a, b);
      boundary_local(k, bi, bj);
      gs[idx] = A.u_in[(int64_t)(kHalf * b + bj) * A.pitch + kHalf * a + bi];
    }
    __syncthreads();
    // Thread t owns 4 consecutive columns (group t % (D/4)) and a 16-wide
    // slice of k (t / (D/4)); its 16 float4 weight loads are independent, so
    // they are in flight together. The 8 k-slice partials go to LDS scratch
    // that aliases the activation tile (not in use yet) and are then summed.
    constexpr int NG = D / 4, KSL = NTH / NG, KPS = kNB / KSL;
    static_assert(KSL * KPS == kNB, "projection split");
    static_assert((size_t)KSL * NPMAX * D * sizeof(float) <= sizeof(HT) * R * LDH, "projection scratch");
    const int n4 = tid % NG, ks = tid / NG;
    floatx4 w[KPS];
#pragma unroll
    for (int i = 0; i < KPS; ++i)
      w[i] = *reinterpret_cast<const floatx4*>(net.w1gT + (ks * KPS + i) * D + 4 * n4);
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
      cs[idx] = c;
    }
  }
  __syncthreads();

  // -- first layer: tanh(projection + W1x (x, y)) ---------------------------
  {
    const int n = tid & (D - 1);
    const float wx = net.w1x[2 * n], wy = net.w1x[2 * n + 1];
    const float bb = net.b1[n];
    for (int r = tid / D; r < R; r += NTH / D) {
      float c;
      if constexpr (SRC == SRC_GATHER) {
        c = cs[r_slot[r] * D + n] + bb;
      } else {
        c = A.C[r_bc[r] * D + n];
      }
      const float pre = fmaf(r_y[r], wy, fmaf(r_x[r], wx, c));
      h_store<PREC>(&Hs[r * LDH + n], tanh_fast(pre));
    }
  }
  __syncthreads();

  // -- hidden layers on MFMA --------------------------------------------------
  if constexpr (PREC == 1) {
    hidden_layers_bf16<D, R, CPW>(Hs, static_cast<const u32x4*>(net.wh), net.bh, lane, wave);
  } else if constexpr (R >= 64) {
    hidden_layers_f32<D, R>(Hs, static_cast<const floatx4*>(net.wh), net.bh, lane, wave);
  } else {
    const int arow = lane & 31;
    for (int l = 0; l < 3; ++l) {
      floatx16 acc[RB];
      mfma_layer_f32<D, RB, LDH>(Hs, static_cast<const floatx4*>(net.wh) + (size_t)l * (D * D / 4) +
                                         (size_t)wave * (D / 8) * 64 + lane,
                                 acc, lane);
      __syncthreads();   // every wave has finished reading this layer's input
      const int j = wave * 32 + arow;
      const float bj = net.bh[l * D + j];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int i = rb * 32 + acc_row(lane, v);
          Hs[i * LDH + j] = tanh_fast(acc[rb][v] + bj);
        }
      __syncthreads();
    }
  }

  // -- output layer and store -------------------------------------------------
  // Eight threads per row, whatever the tile height, so a row's dot product
  // is summed in the same order for every tile shape.
  {
    constexpr int TPR = 8;
    const int part = tid % TPR;
    for (int r = tid / TPR; r < R; r += NTH / TPR) {
      float s = 0.0f;
      for (int n = part; n < D; n += TPR) s = fmaf(h_load<PREC>(&Hs[r * LDH + n]), net.w5[n], s);
#pragma unroll
      for (int o = TPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (part == 0) {
        const int64_t addr = r_addr[r];
        if (addr >= 0) {
          const float val = s + net.b5[0];
          if constexpr (OUT == OUT_STORE) A.u_out[addr] = val;
          else if constexpr (OUT == OUT_ACCUM) A.u_out[addr] += val * r_w[r];
          else A.U[addr] = val;
        }
      }
    }
  }
}

template <int D, int R, int TMODE, int PREC, int SRC, int OUT, int CPW = 32>
__global__ __launch_bounds__((D / CPW) * 64) void tile_kernel(TileArgs A) {
  tile_body<D, R, TMODE, PREC, SRC, OUT, CPW>(A, (int64_t)blockIdx.x * R);
}

// Batched independent domains in one persistent launch per colour: block b
// takes tiles b, b + gridDim.x, ...; tile t belongs to the domain d with
// tile_begin[d] <= t < tile_begin[d + 1] and covers rows
// [(t - tile_begin[d]) R, ... + R) of that domain's phase.
struct MultiArgs {
  TileArgs base;             // network; colour
  const float* field_in;     // packed fields (domain offsets are relative to these)
  float* field_out;
  const DomEntry* doms;      // [n_domains]
  const int32_t* tile_begin; // [n_domains + 1] for this colour and target set
  int n_domains;
  int64_t n_tiles;
};

template <int D, int R, int TMODE, int PREC, int OUT, int CPW = 32>
__global__ __launch_bounds__((D / CPW) * 64) void tile_kernel_multi(MultiArgs M) {
  constexpr int T = n_targets<TMODE>();
  const int ca = M.base.colour & 1, cb = M.base.colour >> 1;
  for (int64_t t = blockIdx.x; t < M.n_tiles; t += gridDim.x) {
    int lo = 0, hi = M.n_domains - 1;       // last d with tile_begin[d] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (M.tile_begin[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const DomEntry e = M.doms[lo];
    TileArgs A = M.base;
    A.u_in = M.field_in + e.offset;
    A.u_out = M.field_out + e.offset;
    A.pitch = e.pitch;
    A.ux = e.ux;
    A.uy = e.uy;
    A.total_rows = (int64_t)(e.ux - ca) * (e.uy - cb) * T;
    tile_body<D, R, TMODE, PREC, SRC_GATHER, OUT, CPW>(A, (t - M.tile_begin[lo]) * R);
    __syncthreads();   // the next tile reuses the LDS
  }
}

template <int D, int R, int TMODE, int PREC, int OUT, int CPW = 32>
static hipError_t launch_multi(const MultiArgs& m, int n_cu, hipStream_t s) {
  if (m.n_tiles == 0) return hipSuccess;
  constexpr int NTH = (D / CPW) * 64;
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tile_kernel_multi<D, R, TMODE, PREC, OUT, CPW>,
                                                     NTH, 0) != hipSuccess || nb < 1)
      nb = 1;
    per_cu = nb;
  }
  const int64_t grid = std::min<int64_t>(m.n_tiles, (int64_t)per_cu * n_cu);
  hipLaunchKernelGGL((tile_kernel_multi<D, R, TMODE, PREC, OUT, CPW>), dim3((unsigned)grid), dim3(NTH), 0,
                     s, m);
  return hipGetLastError();
}

template <int D, int R, int PREC, int CPW = 32>
static hipError_t dispatch_multi(const MultiArgs& m, int targets, bool accumulate, int n_cu,
                                 hipStream_t s) {
  if (accumulate)
    return targets == MF_CROSS ? launch_multi<D, R, 0, PREC, OUT_ACCUM, CPW>(m, n_cu, s)
                               : launch_multi<D, R, 1, PREC, OUT_ACCUM, CPW>(m, n_cu, s);
  if (targets == MF_CROSS) return launch_multi<D, R, 0, PREC, OUT_STORE, CPW>(m, n_cu, s);
  return launch_multi<D, R, 1, PREC, OUT_STORE, CPW>(m, n_cu, s);
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
  if (prec == MF_BF16 && (tile_rows & MF_TILE_WIDE)) {
    const int r = tile_rows & ~MF_TILE_WIDE;
    if (width == 256)
      return r == 256 ? dispatch_multi<256, 256, 1, 64>(m, targets, accumulate, n_cu, s)
                      : dispatch_multi<256, 128, 1, 64>(m, targets, accumulate, n_cu, s);
    return r == 256 ? dispatch_multi<128, 256, 1, 64>(m, targets, accumulate, n_cu, s)
                    : dispatch_multi<128, 128, 1, 64>(m, targets, accumulate, n_cu, s);
  }
  if (prec == MF_BF16) {
    if (width == 256) {
      if (tile_rows == 256) return dispatch_multi<256, 256, 1>(m, targets, accumulate, n_cu, s);
      if (tile_rows == 128) return dispatch_multi<256, 128, 1>(m, targets, accumulate, n_cu, s);
      return dispatch_multi<256, 64, 1>(m, targets, accumulate, n_cu, s);
    }
    if (tile_rows == 256) return dispatch_multi<128, 256, 1>(m, targets, accumulate, n_cu, s);
    if (tile_rows == 128) return dispatch_multi<128, 128, 1>(m, targets, accumulate, n_cu, s);
    return dispatch_multi<128, 64, 1>(m, targets, accumulate, n_cu, s);
  }
  if (width == 256)
    return tile_rows == 64 ? dispatch_multi<256, 64, 0>(m, targets, accumulate, n_cu, s)
                           : dispatch_multi<256, 32, 0>(m, targets, accumulate, n_cu, s);
  return tile_rows == 64 ? dispatch_multi<128, 64, 0>(m, targets, accumulate, n_cu, s)
                         : dispatch_multi<128, 32, 0>(m, targets, accumulate, n_cu, s);
}

template <int D, int R, int TMODE, int PREC, int SRC, int OUT, int CPW = 32>
static hipError_t launch_tile(const TileArgs& a, hipStream_t s) {
  const int64_t blocks = (a.total_rows + R - 1) / R;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((tile_kernel<D, R, TMODE, PREC, SRC, OUT, CPW>), dim3((unsigned)blocks),
                     dim3((D / CPW) * 64), 0, s, a);
  return hipGetLastError();
}

template <int D, int R, int PREC, int CPW = 32>
static hipError_t dispatch_phase(const TileArgs& a, int targets, bool accumulate, hipStream_t s) {
  if (accumulate)
    return targets == MF_CROSS ? launch_tile<D, R, 0, PREC, SRC_GATHER, OUT_ACCUM, CPW>(a, s)
                               : launch_tile<D, R, 1, PREC, SRC_GATHER, OUT_ACCUM, CPW>(a, s);
  if (targets == MF_CROSS) return launch_tile<D, R, 0, PREC, SRC_GATHER, OUT_STORE, CPW>(a, s);
  return launch_tile<D, R, 1, PREC, SRC_GATHER, OUT_STORE, CPW>(a, s);
}

static int64_t colour_count(int ux, int uy, int colour) {
  return (int64_t)(ux - (colour & 1)) * (uy - (colour >> 1));
}

int pick_tile_rows(int width, int prec, int targets, int64_t rows, int n_cu) {
  (void)width; (void)targets;
  if (prec == MF_BF16) {
    if (rows >= (int64_t)256 * 3 * n_cu) return 256;
    if (rows >= (int64_t)128 * 2 * n_cu) return 128;
    return 64;
  }
  return rows >= (int64_t)64 * 2 * n_cu ? 64 : 32;
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
  if (prec == MF_BF16 && (tile_rows & MF_TILE_WIDE)) {
    const int r = tile_rows & ~MF_TILE_WIDE;
    if (width == 256)
      return r == 256 ? dispatch_phase<256, 256, 1, 64>(a, targets, accumulate, s)
                      : dispatch_phase<256, 128, 1, 64>(a, targets, accumulate, s);
    return r == 256 ? dispatch_phase<128, 256, 1, 64>(a, targets, accumulate, s)
                    : dispatch_phase<128, 128, 1, 64>(a, targets, accumulate, s);
  }
  if (prec == MF_BF16) {
    if (width == 256) {
      if (tile_rows == 256) return dispatch_phase<256, 256, 1>(a, targets, accumulate, s);
      if (tile_rows == 128) return dispatch_phase<256, 128, 1>(a, targets, accumulate, s);
      return dispatch_phase<256, 64, 1>(a, targets, accumulate, s);
    }
    if (tile_rows == 256) return dispatch_phase<128, 256, 1>(a, targets, accumulate, s);
    if (tile_rows == 128) return dispatch_phase<128, 128, 1>(a, targets, accumulate, s);
    return dispatch_phase<128, 64, 1>(a, targets, accumulate, s);
  }
  if (width == 256)
    return tile_rows == 64 ? dispatch_phase<256, 64, 0>(a, targets, accumulate, s)
                           : dispatch_phase<256, 32, 0>(a, targets, accumulate, s);
  return tile_rows == 64 ? dispatch_phase<128, 64, 0>(a, targets, accumulate, s)
                         : dispatch_phase<128, 32, 0>(a, targets, accumulate, s);
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
  if (width == 256)
    return prec == MF_FP32 ? launch_tile<256, 64, 0, 0, SRC_C, OUT_LINEAR>(a, s)
                           : launch_tile<256, 64, 0, 1, SRC_C, OUT_LINEAR>(a, s);
  return prec == MF_FP32 ? launch_tile<128, 64, 0, 0, SRC_C, OUT_LINEAR>(a, s)
                         : launch_tile<128, 64, 0, 1, SRC_C, OUT_LINEAR>(a, s);
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
__global__ __launch_bounds__(256) void operator_kernel(const float* __restrict__ Hop, PhaseArgs p) {
  constexpr int T = n_targets<TMODE>();
  __shared__ float g[kNB];
  int a, b;
  placement_of(blockIdx.x, p.colour, p.ux, a, b);
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
  if (n == 0) return hipSuccess;
  if (accumulate)
    hipLaunchKernelGGL((operator_kernel<1, OUT_ACCUM>), dim3((unsigned)n), dim3(256), 0, s, Hop, p);
  else if (targets == MF_CROSS)
    hipLaunchKernelGGL((operator_kernel<0, OUT_STORE>), dim3((unsigned)n), dim3(256), 0, s, Hop, p);
  else
    hipLaunchKernelGGL((operator_kernel<1, OUT_STORE>), dim3((unsigned)n), dim3(256), 0, s, Hop, p);
  return hipGetLastError();
}

}  // namespace mf

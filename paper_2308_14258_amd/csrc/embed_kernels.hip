// The paper's SDNet architecture on gfx950 (Sec. 3.1, Fig. 3): a circular
// 1-D convolutional embedding of each boundary curve, the input-split first
// layer on that embedding (Sec. 3.2, Eq. 8) and GELU layers.
//
// Per boundary condition (a training condition, or a placement of a colour
// phase whose boundary is gathered from the field), one workgroup computes
//   h1 = GELU(conv1(g)), e = GELU(conv2(h1))  (circular, kernel 5, C channels)
//   c  = W1e e + b1                            (E = 128 C inputs, d outputs)
// once, staged in LDS; every point of the condition then starts from c
// (fwd_layer1_kernel with the GELU rules), the three hidden layers run on
// MFMA (taylor_gemm_kernel with the GELU epilogue) and the output layer
// stores, scatters or overlap-averages the value (rows_output_kernel).
#include <algorithm>

#include "mf_device.h"
#include "mf_internal.h"

namespace mf {

// Transposed embedding block of W1 ([E][d], coalesced over the output unit)
// from the flat parameters (W1 of shape d x (E + 2) at offset w1_off).
__global__ void prepare_w1eT_kernel(const float* __restrict__ params, int64_t w1_off, int d, int E,
                                    float* __restrict__ w1eT) {
  const int64_t n = (int64_t)E * d;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / d, j = idx - i * d;
    w1eT[idx] = params[w1_off + j * (E + 2) + i];
  }
}

// One workgroup per boundary condition b (256 threads). SRC 0: g = G[b];
// SRC 1: g = the boundary of placement q0 + b of the colour, gathered from
// the field. conv: the C x 1 x 5 and C x C x 5 weights and biases at the
// start of the flat parameters.
template <int D, int SRC>
__global__ __launch_bounds__(256) void embed_project_kernel(const float* __restrict__ conv, int C,
                                                            const float* __restrict__ w1eT,
                                                            const float* __restrict__ b1,
                                                            const float* __restrict__ G,
                                                            const float* __restrict__ u, int64_t pitch, int ux,
                                                            int colour, int q0, float* __restrict__ Cout) {
  extern __shared__ float sm[];   // g [128] | h1 [C][128] | e [C][128]
  float* g = sm;
  float* h1 = sm + kNB;
  float* e = h1 + C * kNB;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (tid < kNB) {
    if constexpr (SRC == 0) {
      g[tid] = G[(int64_t)b * kNB + tid];
    } else {
      int a, bb, bi, bj;
      placement_of(q0 + b, colour, ux, a, bb);
      boundary_local(tid, bi, bj);
      g[tid] = u[(int64_t)(kHalf * bb + bj) * pitch + kHalf * a + bi];
    }
  }
  __syncthreads();
  const float* w1c = conv;
  const float* b1c = w1c + C * kConvK;
  const float* w2c = b1c + C;
  const float* b2c = w2c + C * C * kConvK;
  for (int idx = tid; idx < C * kNB; idx += 256) {
    const int o = idx >> 7, k = idx & 127;
    float acc = b1c[o];
#pragma unroll
    for (int t = 0; t < kConvK; ++t) acc = fmaf(w1c[o * kConvK + t], g[(k + t - 2) & 127], acc);
    h1[idx] = gelu_f32(acc);
  }
  __syncthreads();
  for (int idx = tid; idx < C * kNB; idx += 256) {
    const int o = idx >> 7, k = idx & 127;
    float acc = b2c[o];
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int t = 0; t < kConvK; ++t) acc = fmaf(w2c[(o * C + i) * kConvK + t], h1[i * kNB + ((k + t - 2) & 127)], acc);
    e[idx] = gelu_f32(acc);
  }
  __syncthreads();
  const int E = C * kNB;
  for (int j = tid; j < D; j += 256) {
    float acc = 0.0f;
    for (int i = 0; i < E; ++i) acc = fmaf(w1eT[(int64_t)i * D + j], e[i], acc);
    Cout[(int64_t)b * D + j] = acc + b1[j];
  }
}

// Reverse of the embedding for the training gradient. One workgroup per
// condition b recomputes p1 = conv1(g) + bc1, h1 = GELU(p1) and
// p2 = conv2(h1) + bc2 in LDS. MODE 0 writes e = GELU(p2) ([B][128 C], the
// first layer's input columns). MODE 1 takes the first layer's
// per-condition sums of the pre-activation adjoint from the two passes,
// c = c0[b] + c1[b], forms e_bar = W1e^T c, then p2_bar = e_bar GELU'(p2),
// the second convolution's kernel and bias gradients, h1_bar (the circular
// convolution transposed), p1_bar = h1_bar GELU'(p1) and the first
// convolution's gradients, into part[b][0 .. 10 C + 5 C^2) in the order of
// the parameters. Every sum runs in a fixed order.
template <int MODE>
__global__ __launch_bounds__(256) void embed_grad_kernel(const float* __restrict__ conv, int C,
                                                         const float* __restrict__ w1, int d,
                                                         const float* __restrict__ G, const float* __restrict__ c0,
                                                         const float* __restrict__ c1, float* __restrict__ e_out,
                                                         float* __restrict__ part) {
  extern __shared__ float sm[];   // g [128] | p1, h1, p2, v [C][128] each | c [d]
  const int E = C * kNB;
  float* g = sm;
  float* p1 = g + kNB;
  float* h1 = p1 + E;
  float* p2 = h1 + E;
  float* v = p2 + E;
  float* cs = v + E;
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < kNB) g[tid] = G[b * kNB + tid];
  __syncthreads();
  const float* w1c = conv;
  const float* b1c = w1c + C * kConvK;
  const float* w2c = b1c + C;
  const float* b2c = w2c + C * C * kConvK;
  for (int idx = tid; idx < E; idx += 256) {
    const int o = idx >> 7, k = idx & 127;
    float acc = b1c[o];
#pragma unroll
    for (int t = 0; t < kConvK; ++t) acc = fmaf(w1c[o * kConvK + t], g[(k + t - 2) & 127], acc);
    p1[idx] = acc;
    h1[idx] = gelu_f32(acc);
  }
  __syncthreads();
  for (int idx = tid; idx < E; idx += 256) {
    const int o = idx >> 7, k = idx & 127;
    float acc = b2c[o];
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int t = 0; t < kConvK; ++t) acc = fmaf(w2c[(o * C + i) * kConvK + t], h1[i * kNB + ((k + t - 2) & 127)], acc);
    p2[idx] = acc;
  }
  __syncthreads();
  if constexpr (MODE == 0) {
    for (int idx = tid; idx < E; idx += 256) e_out[b * E + idx] = gelu_f32(p2[idx]);
    return;
  }
  for (int j = tid; j < d; j += 256) cs[j] = c0[b * d + j] + c1[b * d + j];
  __syncthreads();
  for (int idx = tid; idx < E; idx += 256) {   // p2_bar = (W1e^T c) GELU'(p2)
    float eb = 0.0f;
    for (int j = 0; j < d; ++j) eb = fmaf(w1[(int64_t)j * (E + 2) + idx], cs[j], eb);
    float z, d1, d2;
    gelu_rules(p2[idx], z, d1, d2);
    v[idx] = eb * d1;
  }
  __syncthreads();
  float* P = part + b * (int64_t)(2 * C + C * kConvK + C * C * kConvK);
  float* P2 = P + C * kConvK + C;   // the second convolution's kernel, then its bias
  for (int q = tid; q < C * C * kConvK; q += 256) {
    const int o = q / (C * kConvK), i = (q / kConvK) % C, t = q % kConvK;
    float acc = 0.0f;
    for (int k = 0; k < kNB; ++k) acc = fmaf(v[o * kNB + k], h1[i * kNB + ((k + t - 2) & 127)], acc);
    P2[q] = acc;
  }
  for (int o = tid; o < C; o += 256) {
    float acc = 0.0f;
    for (int k = 0; k < kNB; ++k) acc += v[o * kNB + k];
    P2[C * C * kConvK + o] = acc;
  }
  for (int idx = tid; idx < E; idx += 256) {   // p1_bar = h1_bar GELU'(p1), into p2's space
    const int i = idx >> 7, m = idx & 127;
    float hb = 0.0f;
    for (int o = 0; o < C; ++o)
#pragma unroll
      for (int t = 0; t < kConvK; ++t) hb = fmaf(w2c[(o * C + i) * kConvK + t], v[o * kNB + ((m - t + 2) & 127)], hb);
    float z, d1, d2;
    gelu_rules(p1[idx], z, d1, d2);
    p2[idx] = hb * d1;
  }
  __syncthreads();
  for (int q = tid; q < C * kConvK; q += 256) {
    const int o = q / kConvK, t = q % kConvK;
    float acc = 0.0f;
    for (int k = 0; k < kNB; ++k) acc = fmaf(p2[o * kNB + k], g[(k + t - 2) & 127], acc);
    P[q] = acc;
  }
  for (int o = tid; o < C; o += 256) {
    float acc = 0.0f;
    for (int k = 0; k < kNB; ++k) acc += p2[o * kNB + k];
    P[C * kConvK + o] = acc;
  }
}

// Boundary adjoint of the GELU network for the sweep's adjoint: per placement
// q (one workgroup), c = the first layer's pre-activation adjoint sum over
// the placement's targets, e_bar = W1e^T c (w1eT: the transposed block,
// [E][d]), then back through the two convolutions as in embed_grad_kernel,
// ending at the boundary values: g_bar[m] = sum_o sum_t Wc1[o][t]
// p1_bar[o][(m - t + 2) mod 128].
__global__ __launch_bounds__(256) void embed_input_adjoint_kernel(const float* __restrict__ conv, int C,
                                                                  const float* __restrict__ w1eT, int d,
                                                                  const float* __restrict__ G,
                                                                  const float* __restrict__ c,
                                                                  float* __restrict__ gb) {
  extern __shared__ float sm[];   // g [128] | p1, h1, p2, v [C][128] each | c [d]
  const int E = C * kNB;
  float* g = sm;
  float* p1 = g + kNB;
  float* h1 = p1 + E;
  float* p2 = h1 + E;
  float* v = p2 + E;
  float* cs = v + E;
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < kNB) g[tid] = G[q * kNB + tid];
  for (int j = tid; j < d; j += 256) cs[j] = c[q * d + j];
  __syncthreads();
  const float* w1c = conv;
  const float* b1c = w1c + C * kConvK;
  const float* w2c = b1c + C;
  const float* b2c = w2c + C * C * kConvK;
  for (int idx = tid; idx < E; idx += 256) {
    const int o = idx >> 7, k = idx & 127;
    float acc = b1c[o];
#pragma unroll
    for (int t = 0; t < kConvK; ++t) acc = fmaf(w1c[o * kConvK + t], g[(k + t - 2) & 127], acc);
    p1[idx] = acc;
    h1[idx] = gelu_f32(acc);
  }
  __syncthreads();
  for (int idx = tid; idx < E; idx += 256) {
    const int o = idx >> 7, k = idx & 127;
    float acc = b2c[o];
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int t = 0; t < kConvK; ++t) acc = fmaf(w2c[(o * C + i) * kConvK + t], h1[i * kNB + ((k + t - 2) & 127)], acc);
    p2[idx] = acc;
  }
  __syncthreads();
  for (int idx = tid; idx < E; idx += 256) {   // p2_bar = (W1e^T c) GELU'(p2)
    float eb = 0.0f;
    for (int j = 0; j < d; ++j) eb = fmaf(w1eT[(int64_t)idx * d + j], cs[j], eb);
    float z, d1, d2;
    gelu_rules(p2[idx], z, d1, d2);
    v[idx] = eb * d1;
  }
  __syncthreads();
  for (int idx = tid; idx < E; idx += 256) {   // p1_bar = h1_bar GELU'(p1), into p2's space
    const int i = idx >> 7, m = idx & 127;
    float hb = 0.0f;
    for (int o = 0; o < C; ++o)
#pragma unroll
      for (int t = 0; t < kConvK; ++t) hb = fmaf(w2c[(o * C + i) * kConvK + t], v[o * kNB + ((m - t + 2) & 127)], hb);
    float z, d1, d2;
    gelu_rules(p1[idx], z, d1, d2);
    p2[idx] = hb * d1;
  }
  __syncthreads();
  if (tid < kNB) {
    float acc = 0.0f;
    for (int o = 0; o < C; ++o)
#pragma unroll
      for (int t = 0; t < kConvK; ++t) acc = fmaf(w1c[o * kConvK + t], p2[o * kNB + ((tid - t + 2) & 127)], acc);
    gb[q * kNB + tid] = acc;
  }
}

hipError_t launch_embed_input_adjoint(const float* params, const NetPtrs& net, int width, int C, const float* G,
                                      const float* c, int n_q, float* gb, hipStream_t s) {
  const size_t lds = (size_t)(kNB + 4 * C * kNB + width) * 4;
  hipLaunchKernelGGL(embed_input_adjoint_kernel, dim3((unsigned)n_q), dim3(256), lds, s, params, C, net.w1gT, width,
                     G, c, gb);
  return hipGetLastError();
}

hipError_t launch_embed_grad(const float* params, int width, int C, int64_t off_w1, const float* G, int64_t B,
                             const float* c0, const float* c1, float* e_out, float* part, hipStream_t s) {
  const size_t lds = (size_t)(kNB + 4 * C * kNB + width) * 4;
  if (e_out)
    hipLaunchKernelGGL((embed_grad_kernel<0>), dim3((unsigned)B), dim3(256), lds, s, params, C, params + off_w1,
                       width, G, c0, c1, e_out, part);
  else
    hipLaunchKernelGGL((embed_grad_kernel<1>), dim3((unsigned)B), dim3(256), lds, s, params, C, params + off_w1,
                       width, G, c0, c1, e_out, part);
  return hipGetLastError();
}

// Output layer on value rows Z [n_rows][D]: u = w5 . z + b5, one wave per
// row. MODE 0: U[r0 + r] = u. MODE 1: the field at target t of placement
// q0 + r / T of the colour takes u. MODE 2: u_out there += u / cover count.
template <int D, int TMODE, int MODE>
__global__ __launch_bounds__(256) void rows_output_kernel(const float* __restrict__ Z, const float* __restrict__ w5,
                                                          const float* __restrict__ b5, int64_t n_rows,
                                                          float* __restrict__ out, int64_t pitch, int ux, int uy,
                                                          int colour, int q0) {
  constexpr int NJ = D / 64;
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = gw; r < n_rows; r += nw) {
    float p = 0.0f;
#pragma unroll
    for (int t = 0; t < NJ; ++t) p = fmaf(w5[lane + 64 * t], Z[r * D + lane + 64 * t], p);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off);
    if (lane == 0) {
      const float val = p + b5[0];
      if constexpr (MODE == 0) {
        out[r] = val;
      } else {
        constexpr int T = n_targets<TMODE>();
        const int q = (int)(r / T), t = (int)(r - (int64_t)q * T);
        int a, b, ti, tj;
        placement_of(q0 + q, colour, ux, a, b);
        target_local<TMODE>(t, ti, tj);
        const int gi = kHalf * a + ti, gj = kHalf * b + tj;
        const int64_t o = (int64_t)gj * pitch + gi;
        if constexpr (MODE == 1) out[o] = val;
        else out[o] += val * cover_inv(gi, kS * ux) * cover_inv(gj, kS * uy);
      }
    }
  }
}

static int grid_of(int64_t n, int block, int cap = 8192) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, cap));
}

int64_t embed_param_offset(int C) { return (int64_t)C * kConvK + C + (int64_t)C * C * kConvK + C; }

hipError_t launch_prepare_w1eT(const float* params, int width, int C, float* w1eT, hipStream_t s) {
  const int E = C * kNB;
  hipLaunchKernelGGL(prepare_w1eT_kernel, dim3(grid_of((int64_t)E * width, 256, 2048)), dim3(256), 0, s, params,
                     embed_param_offset(C), width, E, w1eT);
  return hipGetLastError();
}

template <int D>
static hipError_t embed_d(const float* params, int C, const NetPtrs& net, const float* G, int64_t n_bc,
                          const float* u, int64_t pitch, int ux, int colour, int q0, float* Cout, hipStream_t s) {
  const size_t lds = (size_t)(kNB + 2 * C * kNB) * sizeof(float);
  if (G)
    hipLaunchKernelGGL((embed_project_kernel<D, 0>), dim3((unsigned)n_bc), dim3(256), lds, s, params, C, net.w1gT,
                       net.b1, G, nullptr, 0, 0, 0, 0, Cout);
  else
    hipLaunchKernelGGL((embed_project_kernel<D, 1>), dim3((unsigned)n_bc), dim3(256), lds, s, params, C, net.w1gT,
                       net.b1, nullptr, u, pitch, ux, colour, q0, Cout);
  return hipGetLastError();
}

// Embeddings and first-layer projections of n_bc conditions: from G
// [n_bc][128] when G is given, else of placements q0 .. q0 + n_bc - 1 of a
// colour gathered from the field u. Cout: [n_bc][width].
hipError_t launch_embed_project(const float* params, int width, int C, const NetPtrs& net, const float* G,
                                int64_t n_bc, const float* u, int64_t pitch, int ux, int colour, int q0,
                                float* Cout, hipStream_t s) {
  return width == 256 ? embed_d<256>(params, C, net, G, n_bc, u, pitch, ux, colour, q0, Cout, s)
                      : embed_d<128>(params, C, net, G, n_bc, u, pitch, ux, colour, q0, Cout, s);
}

template <int D, int TMODE>
static hipError_t rows_out_d(const NetPtrs& net, const float* Z, int64_t n_rows, int mode, float* out,
                             int64_t pitch, int ux, int uy, int colour, int q0, hipStream_t s) {
  const int blocks = grid_of(n_rows, 4, 8192);
  if (mode == 0)
    hipLaunchKernelGGL((rows_output_kernel<D, TMODE, 0>), dim3(blocks), dim3(256), 0, s, Z, net.w5, net.b5, n_rows,
                       out, pitch, ux, uy, colour, q0);
  else if (mode == 1)
    hipLaunchKernelGGL((rows_output_kernel<D, TMODE, 1>), dim3(blocks), dim3(256), 0, s, Z, net.w5, net.b5, n_rows,
                       out, pitch, ux, uy, colour, q0);
  else
    hipLaunchKernelGGL((rows_output_kernel<D, TMODE, 2>), dim3(blocks), dim3(256), 0, s, Z, net.w5, net.b5, n_rows,
                       out, pitch, ux, uy, colour, q0);
  return hipGetLastError();
}

// Output layer of value rows: mode 0 linear into out, 1 stored at the
// targets of a colour chunk, 2 overlap-averaged into out (assembly).
hipError_t launch_rows_output(const NetPtrs& net, int width, int targets, const float* Z, int64_t n_rows, int mode,
                              float* out, int64_t pitch, int ux, int uy, int colour, int q0, hipStream_t s) {
  if (width == 256)
    return targets == MF_INTERIOR ? rows_out_d<256, 1>(net, Z, n_rows, mode, out, pitch, ux, uy, colour, q0, s)
                                  : rows_out_d<256, 0>(net, Z, n_rows, mode, out, pitch, ux, uy, colour, q0, s);
  return targets == MF_INTERIOR ? rows_out_d<128, 1>(net, Z, n_rows, mode, out, pitch, ux, uy, colour, q0, s)
                                : rows_out_d<128, 0>(net, Z, n_rows, mode, out, pitch, ux, uy, colour, q0, s);
}

}  // namespace mf

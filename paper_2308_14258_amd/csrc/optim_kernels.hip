// LAMB, the large-batch optimiser of the SDNet training (Sec. 5.2,
// "Hyperparameters"; You et al., ICLR 2020), as one fused kernel.
//
// One workgroup per parameter tensor ("layer"): it updates the tensor's
// Adam moments, forms the update u = m_hat / (sqrt(v_hat) + eps) + lambda w
// and the two norms ||w_s|| and ||u_s|| in the same pass, reduces them in a
// fixed order (so the step is deterministic), and applies
// w_s -= lr r_s u_s with the trust ratio r_s = ||w_s|| / ||u_s|| (1 when a
// norm is zero or the ratio is switched off) in a second pass over the
// tensor, recomputing u from the moments it wrote. With global-norm
// clipping every workgroup first sums the squared gradient over all tensors
// in the same order, so all of them scale by the same factor without a
// second launch. A whole tensor goes through one CU, so the step is bound by
// that CU's memory traffic (13-24 us for the width-128 network's 66,433
// parameters, depending on whether the tensors are still in the die's L2).
#include "mf_device.h"
#include "mf_internal.h"

namespace mf {

namespace {

constexpr int kLambThreads = 1024, kLambIlp = 4;

// Sum over the workgroup in a fixed order; every thread receives the sum.
// `red` holds kLambThreads / 64 floats; the call starts and ends with a
// barrier, so consecutive calls may reuse it.
__device__ float block_sum(float x, float* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  float t = 0.0f;
  for (int w = 0; w < kLambThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// The update direction m_hat / (sqrt(v_hat) + eps) + lambda w. The bias
// corrections come in as reciprocals and the square root and reciprocal are
// the hardware's (about one ulp each): with a whole tensor on one workgroup
// the kernel is bound by its per-element VALU work, which the correctly
// rounded division and square root sequences roughly quadrupled.
__device__ __forceinline__ float lamb_direction(float mk, float vk, float wk, const LambParams& h) {
  const float den = __builtin_amdgcn_sqrtf(vk * h.ibc2) + h.eps;
  return fmaf(h.wd, wk, mk * h.ibc1 * __builtin_amdgcn_rcpf(den));
}

// Each loop below takes its elements in groups of kLambIlp strides, with all
// of a group's loads issued before its arithmetic, then a plain tail: one
// dependent load per iteration left the kernel waiting on L2 latency. Element
// i of a tensor belongs to thread (i - begin) mod kLambThreads in every loop,
// so the second pass reads the moments the same thread wrote in the first.
__global__ __launch_bounds__(kLambThreads) void lamb_kernel(float* __restrict__ p, float* __restrict__ m,
                                                            float* __restrict__ v, const float* __restrict__ g,
                                                            int64_t n, LambSegments S, LambParams h) {
  constexpr int T = kLambThreads, U = kLambIlp;
  __shared__ float red[kLambThreads / 64];
  const int64_t a = S.begin[blockIdx.x], b = S.begin[blockIdx.x + 1];
  float c = 1.0f;
  if (h.max_grad_norm > 0.0f) {
    float acc[2 * U];
#pragma unroll
    for (int j = 0; j < 2 * U; ++j) acc[j] = 0.0f;
    int64_t i = threadIdx.x;
    for (; i + (2 * U - 1) * T < n; i += 2 * U * T) {
      float gv[2 * U];
#pragma unroll
      for (int j = 0; j < 2 * U; ++j) gv[j] = g[i + j * T];
#pragma unroll
      for (int j = 0; j < 2 * U; ++j) acc[j] = fmaf(gv[j], gv[j], acc[j]);
    }
    for (; i < n; i += T) acc[0] = fmaf(g[i], g[i], acc[0]);
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 2 * U; ++j) s += acc[j];
    const float norm = sqrtf(block_sum(s, red));
    if (norm > h.max_grad_norm) c = h.max_grad_norm / norm;
  }
  float sw = 0.0f, su = 0.0f;
  auto moments = [&](int64_t k, float gk, float wk, float mk, float vk) {
    const float gi = c * gk;
    const float mi = h.b1 * mk + h.omb1 * gi;
    const float vi = h.b2 * vk + h.omb2 * gi * gi;
    m[k] = mi;
    v[k] = vi;
    const float u = lamb_direction(mi, vi, wk, h);
    sw = fmaf(wk, wk, sw);
    su = fmaf(u, u, su);
  };
  int64_t i = a + threadIdx.x;
  for (; i + (U - 1) * T < b; i += U * T) {
    float gv[U], wv[U], mv[U], vv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      gv[j] = g[i + j * T];
      wv[j] = p[i + j * T];
      mv[j] = m[i + j * T];
      vv[j] = v[i + j * T];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) moments(i + j * T, gv[j], wv[j], mv[j], vv[j]);
  }
  for (; i < b; i += T) moments(i, g[i], p[i], m[i], v[i]);
  const float W = block_sum(sw, red), U2 = block_sum(su, red);
  const float r = (h.trust && W > 0.0f && U2 > 0.0f) ? sqrtf(W) / sqrtf(U2) : 1.0f;
  const float step = h.lr * r;
  auto apply = [&](int64_t k, float wk, float mk, float vk) {
    p[k] = wk - step * lamb_direction(mk, vk, wk, h);
  };
  i = a + threadIdx.x;
  for (; i + (U - 1) * T < b; i += U * T) {
    float wv[U], mv[U], vv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      wv[j] = p[i + j * T];
      mv[j] = m[i + j * T];
      vv[j] = v[i + j * T];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) apply(i + j * T, wv[j], mv[j], vv[j]);
  }
  for (; i < b; i += T) apply(i, p[i], m[i], v[i]);
}

}  // namespace

hipError_t launch_lamb(float* p, float* m, float* v, const float* g, const LambSegments& S, double lr, double b1,
                       double b2, double eps, double wd, double max_grad_norm, bool trust, int64_t step,
                       hipStream_t s) {
  LambParams h;
  h.lr = (float)lr;
  h.b1 = (float)b1;
  h.omb1 = (float)(1.0 - b1);
  h.b2 = (float)b2;
  h.omb2 = (float)(1.0 - b2);
  h.eps = (float)eps;
  h.wd = (float)wd;
  h.ibc1 = (float)(1.0 / (1.0 - pow(b1, (double)step)));
  h.ibc2 = (float)(1.0 / (1.0 - pow(b2, (double)step)));
  h.max_grad_norm = (float)max_grad_norm;
  h.trust = trust ? 1 : 0;
  hipLaunchKernelGGL(lamb_kernel, dim3((unsigned)S.n), dim3(kLambThreads), 0, s, p, m, v, g, S.begin[S.n], S, h);
  return hipGetLastError();
}

}  // namespace mf

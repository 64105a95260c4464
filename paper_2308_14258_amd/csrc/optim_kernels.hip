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
// second launch. The tensors of an SDNet are at most a few hundred
// thousand floats: the step is a few microseconds, bound by its two passes
// over p, m, v and g.
#include "mf_device.h"
#include "mf_internal.h"

namespace mf {

namespace {

constexpr int kLambThreads = 1024;

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

__global__ __launch_bounds__(kLambThreads) void lamb_kernel(float* __restrict__ p, float* __restrict__ m,
                                                            float* __restrict__ v, const float* __restrict__ g,
                                                            int64_t n, LambSegments S, LambParams h) {
  __shared__ float red[kLambThreads / 64];
  const int64_t a = S.begin[blockIdx.x], b = S.begin[blockIdx.x + 1];
  float c = 1.0f;
  if (h.max_grad_norm > 0.0f) {
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += kLambThreads) s = fmaf(g[i], g[i], s);
    const float norm = sqrtf(block_sum(s, red));
    if (norm > h.max_grad_norm) c = h.max_grad_norm / norm;
  }
  float sw = 0.0f, su = 0.0f;
  for (int64_t i = a + threadIdx.x; i < b; i += kLambThreads) {
    const float gi = c * g[i], wi = p[i];
    const float mi = h.b1 * m[i] + h.omb1 * gi;
    const float vi = h.b2 * v[i] + h.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float u = (mi / h.bc1) / (sqrtf(vi / h.bc2) + h.eps) + h.wd * wi;
    sw = fmaf(wi, wi, sw);
    su = fmaf(u, u, su);
  }
  const float W = block_sum(sw, red), U = block_sum(su, red);
  const float r = (h.trust && W > 0.0f && U > 0.0f) ? sqrtf(W) / sqrtf(U) : 1.0f;
  const float step = h.lr * r;
  // each thread revisits the elements it wrote: its own m and v are visible
  for (int64_t i = a + threadIdx.x; i < b; i += kLambThreads) {
    const float wi = p[i];
    const float u = (m[i] / h.bc1) / (sqrtf(v[i] / h.bc2) + h.eps) + h.wd * wi;
    p[i] = wi - step * u;
  }
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
  h.bc1 = (float)(1.0 - pow(b1, (double)step));
  h.bc2 = (float)(1.0 - pow(b2, (double)step));
  h.max_grad_norm = (float)max_grad_norm;
  h.trust = trust ? 1 : 0;
  hipLaunchKernelGGL(lamb_kernel, dim3((unsigned)S.n), dim3(kLambThreads), 0, s, p, m, v, g, S.begin[S.n], S, h);
  return hipGetLastError();
}

}  // namespace mf

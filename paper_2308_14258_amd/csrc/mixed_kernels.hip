// Mixed-precision sweeps: 16-bit colour phases whose predictions are
// corrected by a float32 reference refreshed every few sweeps.
//
// The 16-bit map of a colour phase differs from the float32 map by a
// rounding error that is systematic (it depends on the boundary data, not
// on chance), and the one-level iteration (Alg. 2) amplifies a systematic
// error in its slowest modes instead of damping it. A refresh sweep
// evaluates every phase in float32 and, from the same field state, in 16
// bits, and keeps the difference at each target, corr_c = pred32 - pred16;
// the following 16-bit phases add corr_c to their predictions. The
// correction is exact at the refresh state and changes slowly with the
// field, so the iteration's fixed point follows the float32 one.
//
// These kernels touch a colour's targets only. A batch's placements of one
// colour are numbered consecutively over its domains (qbegin: the colour's
// prefix table, nd + 1 entries), as in the batched adjoint; a domain is
// found by binary search. Buffers in the workspace (tmp, corr) cover the
// span of the caller's field from float `lo` on: index = field index - lo.
#include <algorithm>

#include "mf_device.h"
#include "mf_internal.h"

namespace mf {

namespace {

__device__ __forceinline__ DomEntry find_domain(const DomEntry* doms, const int32_t* qb, int nd, int g, int& lq) {
  int lo = 0, hi = nd - 1;   // last d with qb[d] <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (qb[mid] <= g) lo = mid; else hi = mid - 1;
  }
  lq = g - qb[lo];
  return doms[lo];
}

// MODE 0: corr[a - lo] = u[a] - tmp[a - lo]; MODE 1: u[a] += corr[a - lo],
// for every target a of the colour's placements q0 .. q0 + n_q - 1.
template <int TMODE, int MODE>
__global__ void corr_targets_kernel(float* __restrict__ u, const float* __restrict__ tmp, float* __restrict__ corr,
                                    int64_t lo, const DomEntry* __restrict__ doms, const int32_t* __restrict__ qb,
                                    int nd, int colour, int q0, int n_q) {
  constexpr int T = n_targets<TMODE>();
  const int64_t n = (int64_t)n_q * T;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(idx / T), t = (int)(idx - (int64_t)q * T);
    int lq, a, b, ti, tj;
    const DomEntry e = find_domain(doms, qb, nd, q0 + q, lq);
    placement_of(lq, colour, e.ux, a, b);
    target_local<TMODE>(t, ti, tj);
    const int64_t addr = e.offset + (int64_t)(kHalf * b + tj) * e.pitch + kHalf * a + ti;
    if constexpr (MODE == 0) corr[addr - lo] = u[addr] - tmp[addr - lo];
    else u[addr] += corr[addr - lo];
  }
}

constexpr int64_t kCorrChunk = 1 << 24;   // targets per launch

}  // namespace

hipError_t launch_corr_targets(int targets, int mode, float* u, const float* tmp, float* corr, int64_t lo,
                               const DomEntry* doms, const int32_t* qbegin, int nd, int colour, int64_t n_place,
                               hipStream_t s) {
  const int T = targets == MF_INTERIOR ? 961 : 61;
  const int64_t per = std::max<int64_t>(1, kCorrChunk / T);
  for (int64_t q0 = 0; q0 < n_place; q0 += per) {
    const int nq = (int)std::min<int64_t>(per, n_place - q0);
    const int64_t n = (int64_t)nq * T;
    const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 16384)), block(256);
    if (targets == MF_INTERIOR) {
      if (mode == 0)
        hipLaunchKernelGGL((corr_targets_kernel<1, 0>), grid, block, 0, s, u, tmp, corr, lo, doms, qbegin, nd,
                           colour, (int)q0, nq);
      else
        hipLaunchKernelGGL((corr_targets_kernel<1, 1>), grid, block, 0, s, u, tmp, corr, lo, doms, qbegin, nd,
                           colour, (int)q0, nq);
    } else {
      if (mode == 0)
        hipLaunchKernelGGL((corr_targets_kernel<0, 0>), grid, block, 0, s, u, tmp, corr, lo, doms, qbegin, nd,
                           colour, (int)q0, nq);
      else
        hipLaunchKernelGGL((corr_targets_kernel<0, 1>), grid, block, 0, s, u, tmp, corr, lo, doms, qbegin, nd,
                           colour, (int)q0, nq);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mf

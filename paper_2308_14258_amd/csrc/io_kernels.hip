// Boundary gather and target scatter of one colour phase as kernels of their
// own (Sec. 4.2, Alg. 2: every placement of the colour reads its 128-sample
// boundary from the field, and its predictions are written back at its
// targets). The fused colour-phase kernel does both inside its tile; these
// serve callers that run the SDNet themselves, and they are the pure data
// movement of the phase, bound by HBM bandwidth.
//
// Layout: the field is row-major with `pitch` floats per row; G is
// [n_q][128] (placement-major, boundary samples counter-clockwise); the
// predictions are [n_q][T] in the library's target order. One workgroup
// handles one placement, its threads consecutive samples, so G and the
// predictions stream contiguously; on the field, horizontal edges and
// horizontal target lines are contiguous runs, vertical ones touch one
// element per row (one memory transaction per element: on a row-major field
// the vertical edges dominate the traffic).
#include "mf_device.h"
#include "mf_internal.h"

namespace mf {

namespace {

constexpr int kXcds = 8;   // accelerator dies; workgroup i runs on die i mod 8

// Launches cover at most this many placements (work-items per launch stay
// below 2^32 at 256 threads per placement).
constexpr int64_t kIoChunk = 1 << 22;

// Placement handled by workgroup `blk` of a grid of kXcds * per_xcd groups
// over placements q0 .. q0 + n_q - 1: each die takes one contiguous range,
// so the edges that neighbouring placements share (the right edge of (a, b)
// is the left edge of (a + 2, b); the top edge of (a, b) the bottom edge of
// (a, b + 2)) are read through the same L2. Returns -1 past the end.
__device__ __forceinline__ int64_t xcd_placement(int64_t blk, int64_t per_xcd, int64_t q0, int64_t n_q) {
  const int64_t q = (blk % kXcds) * per_xcd + blk / kXcds;
  return q < n_q ? q0 + q : -1;
}

// One 128-thread workgroup per placement: thread k reads boundary sample k.
__global__ __launch_bounds__(kNB) void gather_colour_kernel(const float* __restrict__ u, int64_t pitch, int ux,
                                                           int colour, int64_t q0, int64_t n_q,
                                                           int64_t per_xcd, float* __restrict__ G) {
  const int64_t q = xcd_placement(blockIdx.x, per_xcd, q0, n_q);
  if (q < 0) return;
  int a, b, bi, bj;
  placement_of((int)q, colour, ux, a, b);
  boundary_local(threadIdx.x, bi, bj);
  G[q * kNB + threadIdx.x] = u[(int64_t)(kHalf * b + bj) * pitch + kHalf * a + bi];
}

// One workgroup per placement: threads stride over its T targets.
template <int TMODE, int NT>
__global__ __launch_bounds__(NT) void scatter_colour_kernel(const float* __restrict__ pred, float* __restrict__ u,
                                                           int64_t pitch, int ux, int colour, int64_t q0,
                                                           int64_t n_q, int64_t per_xcd) {
  constexpr int T = n_targets<TMODE>();
  const int64_t q = xcd_placement(blockIdx.x, per_xcd, q0, n_q);
  if (q < 0) return;
  int a, b;
  placement_of((int)q, colour, ux, a, b);
  float* base = u + (int64_t)(kHalf * b) * pitch + kHalf * a;
  const float* src = pred + q * T;
  // all loads of the thread first, then the stores: the placement's reads are
  // in flight together
  constexpr int NI = (T + NT - 1) / NT;
  float v[NI];
#pragma unroll
  for (int r = 0; r < NI; ++r) {
    const int t = threadIdx.x + r * NT;
    v[r] = t < T ? src[t] : 0.0f;
  }
#pragma unroll
  for (int r = 0; r < NI; ++r) {
    const int t = threadIdx.x + r * NT;
    if (t < T) {
      int ti, tj;
      target_local<TMODE>(t, ti, tj);
      base[(int64_t)tj * pitch + ti] = v[r];
    }
  }
}

int64_t per_xcd_of(int64_t n_q) { return (n_q + kXcds - 1) / kXcds; }

}  // namespace

hipError_t launch_gather_colour(const float* u, int64_t pitch, int ux, int colour, int64_t n_q, float* G,
                                hipStream_t s) {
  for (int64_t q0 = 0; q0 < n_q; q0 += kIoChunk) {
    const int64_t n = n_q - q0 < kIoChunk ? n_q - q0 : kIoChunk;
    const int64_t per = per_xcd_of(n);
    hipLaunchKernelGGL(gather_colour_kernel, dim3((unsigned)(per * kXcds)), dim3(kNB), 0, s, u, pitch, ux,
                       colour, q0, n, per, G);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scatter_colour(const float* pred, int targets, float* u, int64_t pitch, int ux, int colour,
                                 int64_t n_q, hipStream_t s) {
  for (int64_t q0 = 0; q0 < n_q; q0 += kIoChunk) {
    const int64_t n = n_q - q0 < kIoChunk ? n_q - q0 : kIoChunk;
    const int64_t per = per_xcd_of(n);
    const dim3 grid((unsigned)(per * kXcds));
    if (targets == 0)
      hipLaunchKernelGGL((scatter_colour_kernel<0, 64>), grid, dim3(64), 0, s, pred, u, pitch, ux, colour, q0, n,
                         per);
    else
      hipLaunchKernelGGL((scatter_colour_kernel<1, 256>), grid, dim3(256), 0, s, pred, u, pitch, ux, colour, q0,
                         n, per);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mf

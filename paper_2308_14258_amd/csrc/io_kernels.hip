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
#include <algorithm>

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

// ---------------------------------------------------------------------------
// Skeleton side layout. The boundaries every gather reads and the CROSS
// targets every scatter writes are skeleton points: grid rows j = 16 r and
// grid columns i = 16 c. The rows are contiguous in the row-major field;
// the columns are kept transposed in a side buffer, cols[c * cpitch + j] =
// u[j][16 c], so that vertical edges and vertical centre lines are
// contiguous too. Between pack and unpack the state of a CROSS sweep is the
// field's skeleton rows plus cols (the intersections live in both and are
// written to both); the field's own column entries are refreshed by unpack.
// ---------------------------------------------------------------------------

// cols[c][j] = u[j][16 c]; one thread per (c, j), j fastest.
__global__ void skel_pack_kernel(const float* __restrict__ u, int64_t pitch, int nc, int ny, int64_t cpitch,
                                 float* __restrict__ cols) {
  const int64_t n = (int64_t)nc * ny;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / ny, j = idx - c * ny;
    cols[c * cpitch + j] = u[j * pitch + kHalf * c];
  }
}

__global__ void skel_unpack_kernel(const float* __restrict__ cols, int64_t cpitch, int nc, int ny,
                                   float* __restrict__ u, int64_t pitch) {
  const int64_t n = (int64_t)nc * ny;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / ny, j = idx - c * ny;
    u[j * pitch + kHalf * c] = cols[c * cpitch + j];
  }
}

// Gather from the side layout: each of the four edges is one contiguous run
// (bottom and top in the field's rows, right and left in cols). A workgroup
// has PPW placement slots (128 threads each for the gather, 64 for the
// scatter) and each thread handles ILP placements, PPW apart, whose loads it
// issues together: the kernels are bound by the bytes in flight per CU, and
// one 4-byte load per thread leaves the HBM pipe mostly idle.
constexpr int kSkelPPW = 4, kGatherIlp = 8;
constexpr int kScatterPPW = 4, kScatterIlp = 4;
// Placement of slot `sub` of workgroup `blk` (die blk mod 8): each die's
// workgroups walk its contiguous range `group` placements at a time.
__device__ __forceinline__ int64_t xcd_placement_ppw(int64_t blk, int sub, int group, int64_t per_xcd, int64_t q0,
                                                     int64_t n_q) {
  const int64_t q = (blk % kXcds) * per_xcd + (blk / kXcds) * group + sub;
  return q < n_q ? q0 + q : -1;
}
__global__ __launch_bounds__(kNB * kSkelPPW) void gather_skel_kernel(const float* __restrict__ u, int64_t pitch,
                                                          const float* __restrict__ cols, int64_t cpitch, int ux,
                                                          int colour, int64_t q0, int64_t n_q, int64_t per_xcd,
                                                          float* __restrict__ G) {
  const int k = threadIdx.x & 127, side = k >> 5, m = k & 31;
  float v[kGatherIlp];
  int64_t qs[kGatherIlp];
  // addresses formed without branches, so that the loads are in flight
  // together; a slot past the end reads placement q0 and stores nothing
#pragma unroll
  for (int i = 0; i < kGatherIlp; ++i) {
    const int64_t q =
        xcd_placement_ppw(blockIdx.x, (threadIdx.x >> 7) + i * kSkelPPW, kSkelPPW * kGatherIlp, per_xcd, q0, n_q);
    qs[i] = q;
    int a, b;
    placement_of((int)(q >= 0 ? q : q0), colour, ux, a, b);
    const int64_t r0 = (int64_t)kHalf * b;    // bottom row / first row of the vertical edges
    const int mm = side < 2 ? m : kS - m;      // sides 2 and 3 run backwards
    const bool in_u = (side & 1) == 0;         // (m, 0) and (32 - m, 32) in the field; (32, m), (0, 32 - m) in cols
    const int64_t off = in_u ? (r0 + (side == 2 ? kS : 0)) * pitch + kHalf * a + mm
                             : (int64_t)(side == 1 ? a + 2 : a) * cpitch + r0 + mm;
    v[i] = (in_u ? u : cols)[off];
  }
#pragma unroll
  for (int i = 0; i < kGatherIlp; ++i)
    if (qs[i] >= 0) G[qs[i] * kNB + k] = v[i];
}

// CROSS scatter into the side layout: the vertical centre line (targets
// 0..30, j = 1..31) into cols, the horizontal one (targets 31..60) into the
// field's row, and the centre (target 15) into that row as well.
__global__ __launch_bounds__(64 * kScatterPPW) void scatter_skel_kernel(const float* __restrict__ pred,
                                                          float* __restrict__ u,
                                                          int64_t pitch, float* __restrict__ cols, int64_t cpitch,
                                                          int ux, int colour, int64_t q0, int64_t n_q,
                                                          int64_t per_xcd) {
  const int t = threadIdx.x & 63;
  float v[kScatterIlp];
  int64_t qs[kScatterIlp];
  // loads first, without branches (lanes 61..63 and slots past the end read
  // a valid prediction and store nothing or the centre)
#pragma unroll
  for (int i = 0; i < kScatterIlp; ++i) {
    const int64_t q =
        xcd_placement_ppw(blockIdx.x, (threadIdx.x >> 6) + i * kScatterPPW, kScatterPPW * kScatterIlp, per_xcd, q0,
                          n_q);
    qs[i] = q;
    v[i] = pred[(q >= 0 ? q : q0) * kCross + (t < kCross ? t : kHalf - 1)];
  }
#pragma unroll
  for (int i = 0; i < kScatterIlp; ++i) {
    const int64_t q = qs[i];
    if (q < 0) continue;
    int a, b;
    placement_of((int)q, colour, ux, a, b);
    float* row = u + (int64_t)(kHalf * b + kHalf) * pitch + kHalf * a;   // row j = 16 b + 16 from i = 16 a
    if (t < 31) {
      cols[(int64_t)(a + 1) * cpitch + kHalf * b + 1 + t] = v[i];
    } else if (t < kCross) {
      int ti, tj;
      target_local<0>(t, ti, tj);
      row[ti] = v[i];
    } else if (t == kCross) {
      row[kHalf] = v[i];   // the centre, target 15, also in the row
    }
  }
}

}  // namespace

int64_t skel_cols_pitch(int uy) { return ((int64_t)kS * uy + 1 + 31) / 32 * 32; }

hipError_t launch_skel_pack(const float* u, int64_t pitch, int ux, int uy, float* cols, hipStream_t s) {
  const int nc = 2 * ux + 1, ny = kS * uy + 1;
  const int64_t n = (int64_t)nc * ny;
  hipLaunchKernelGGL(skel_pack_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0, s,
                     u, pitch, nc, ny, skel_cols_pitch(uy), cols);
  return hipGetLastError();
}

hipError_t launch_skel_unpack(const float* cols, float* u, int64_t pitch, int ux, int uy, hipStream_t s) {
  const int nc = 2 * ux + 1, ny = kS * uy + 1;
  const int64_t n = (int64_t)nc * ny;
  hipLaunchKernelGGL(skel_unpack_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0,
                     s, cols, skel_cols_pitch(uy), nc, ny, u, pitch);
  return hipGetLastError();
}

hipError_t launch_gather_skel(const float* u, int64_t pitch, const float* cols, int ux, int uy, int colour,
                              int64_t n_q, float* G, hipStream_t s) {
  for (int64_t q0 = 0; q0 < n_q; q0 += kIoChunk) {
    const int64_t n = n_q - q0 < kIoChunk ? n_q - q0 : kIoChunk;
    constexpr int group = kSkelPPW * kGatherIlp;
    const int64_t per = (per_xcd_of(n) + group - 1) / group * group;
    hipLaunchKernelGGL(gather_skel_kernel, dim3((unsigned)(per * kXcds / group)), dim3(kNB * kSkelPPW), 0, s, u,
                       pitch, cols, skel_cols_pitch(uy), ux, colour, q0, n, per, G);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scatter_skel(const float* pred, float* u, int64_t pitch, float* cols, int ux, int uy, int colour,
                               int64_t n_q, hipStream_t s) {
  for (int64_t q0 = 0; q0 < n_q; q0 += kIoChunk) {
    const int64_t n = n_q - q0 < kIoChunk ? n_q - q0 : kIoChunk;
    constexpr int group = kScatterPPW * kScatterIlp;
    const int64_t per = (per_xcd_of(n) + group - 1) / group * group;
    hipLaunchKernelGGL(scatter_skel_kernel, dim3((unsigned)(per * kXcds / group)), dim3(64 * kScatterPPW), 0, s,
                       pred, u, pitch, cols, skel_cols_pitch(uy), ux, colour, q0, n, per);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

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

// Reverse mode of the predictor: u0_bar = (d u_out / d u0)^T u_out_bar, where
// u_out is the overlap-averaged assembly (Alg. 2, final phase) after K
// multiplicative sweeps started from u0 and u_out_bar is a seed given per grid
// point. Without a seed the objective is J = sum over interior grid points of
// u_out^2, i.e. the seed 2 u_out on the interior and 0 on the ring.
//
// A colour phase writes u'[x] = N(g_p(u), t) at the targets x of every
// placement p of the colour and leaves every other point unchanged. Its
// adjoint, given ub' (the adjoint of the field after the phase):
//   1. ubp[p, t] = ub'[x(p, t)], then ub'[x(p, t)] = 0 (targets were
//      overwritten; same-colour targets are never same-colour boundary points,
//      so these two steps do not interact);
//   2. recompute the placement's network forward from the field before the
//      phase and run the value-stream reverse pass down to the first-layer
//      pre-activation adjoint ab1;
//   3. gb_p = W1g^T sum_t ab1[p, t] (input-split first layer, Eq. 8);
//   4. ub[B_p(k)] += gb_p[k] for the 128 boundary points of p. Placements of
//      one colour share boundary edges, so the scatter runs in four
//      sub-colours (a mod 4, b mod 4) whose boundaries are disjoint: the sum
//      is deterministic with no atomics.
// The assembly's adjoint is the same with ubp[p, t] = seed[x] / count(x) and
// no zeroing; the ring of u_out is the ring of u0, so the seed's ring values
// pass straight into u0_bar. Field states are recomputed from checkpoints taken every
// ckpt_every sweeps.
#include <algorithm>

#include "mf_device.h"
#include "mf_internal.h"

namespace mf {

// Local (x, y) of the T targets, row t of X.
template <int TMODE>
__global__ void target_coords_kernel(float* __restrict__ X) {
  constexpr int T = n_targets<TMODE>();
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
    int i, j;
    target_local<TMODE>(t, i, j);
    X[2 * t] = i * (1.0f / kS);
    X[2 * t + 1] = j * (1.0f / kS);
  }
}

// The placements of one colour over all domains of a batch are numbered
// consecutively, domain by domain: domain d holds the indices
// qbegin[d] .. qbegin[d + 1] - 1 (qbegin: the colour's prefix table, nd + 1
// entries). `locate` finds the domain of a global index g and its local index.
// Domain offsets are those of the caller's buffers; a field copy held in the
// workspace starts `shift` floats later in that frame (its index is the
// caller's minus shift).
struct AdjDomains {
  const DomEntry* doms;     // [nd]
  const int32_t* qbegin;    // [4][nd + 1] per-colour placement prefixes
  int nd;
};

__device__ __forceinline__ DomEntry locate(const AdjDomains& D, int colour, int g, int& lq) {
  const int32_t* qb = D.qbegin + colour * (D.nd + 1);
  int lo = 0, hi = D.nd - 1;   // last d with qb[d] <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (qb[mid] <= g) lo = mid; else hi = mid - 1;
  }
  lq = g - qb[lo];
  return D.doms[lo];
}

// Boundary vectors G [n_q][128] of global placements q0 .. q0 + n_q - 1 of a colour.
__global__ void gather_boundaries_kernel(const float* __restrict__ u, int64_t shift, AdjDomains D, int colour,
                                         int q0, int n_q, float* __restrict__ G) {
  const int64_t n = (int64_t)n_q * kNB;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(idx >> 7), k = (int)(idx & 127);
    int lq, a, b, bi, bj;
    const DomEntry e = locate(D, colour, q0 + q, lq);
    placement_of(lq, colour, e.ux, a, b);
    boundary_local(k, bi, bj);
    G[idx] = u[e.offset - shift + (int64_t)(kHalf * b + bj) * e.pitch + kHalf * a + bi];
  }
}

// Target adjoints of placements q0 .. q0 + n_q - 1.
//   MODE 0 (sweep phase):          ubp = ub[x], then ub[x] = 0.
//   MODE 1 (assembly, sum of u^2): ubp = 2 u_out[x] / count(x).
//   MODE 2 (assembly, seed):       ubp = seed[x] / count(x), seed in u_out's place.
template <int TMODE, int MODE>
__global__ void target_adjoint_kernel(float* __restrict__ ub, const float* __restrict__ u_out, int64_t out_shift,
                                      AdjDomains D, int colour, int q0, int n_q, float* __restrict__ ubp) {
  constexpr int T = n_targets<TMODE>();
  const int64_t n = (int64_t)n_q * T;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(idx / T), t = (int)(idx - (int64_t)q * T);
    int lq, a, b, ti, tj;
    const DomEntry e = locate(D, colour, q0 + q, lq);
    const int ux = e.ux, uy = e.uy;
    placement_of(lq, colour, ux, a, b);
    target_local<TMODE>(t, ti, tj);
    const int gi = kHalf * a + ti, gj = kHalf * b + tj;
    const int64_t o = e.offset + (int64_t)gj * e.pitch + gi;
    if constexpr (MODE == 0) {
      ubp[idx] = ub[o];
      ub[o] = 0.0f;
    } else if constexpr (MODE == 1) {
      ubp[idx] = 2.0f * u_out[o - out_shift] * cover_inv(gi, kS * ux) * cover_inv(gj, kS * uy);
    } else {
      ubp[idx] = u_out[o - out_shift] * cover_inv(gi, kS * ux) * cover_inv(gj, kS * uy);
    }
  }
}

// ab4[r][j] = (1 - z4^2) w5[j] ubp[r]: the output layer u = w5 . h4 + b5
// reversed through the last tanh.
template <int D>
__global__ void adjoint_seed_kernel(const float* __restrict__ Z4, const float* __restrict__ w5,
                                    const float* __restrict__ ubp, int64_t n_rows, float* __restrict__ Ab) {
  const int64_t n = n_rows * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / D;
    const int j = (int)(idx - r * D);
    const float z = Z4[idx];
    Ab[idx] = (1.0f - z * z) * w5[j] * ubp[r];
  }
}

// The same seed through the GELU network's last layer: GELU'(a4) w5[j] ubp[r]
// with a4 the saved pre-activations.
template <int D>
__global__ void adjoint_seed_gelu_kernel(const float* __restrict__ A4, const float* __restrict__ w5,
                                         const float* __restrict__ ubp, int64_t n_rows, float* __restrict__ Ab) {
  const int64_t n = n_rows * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / D;
    const int j = (int)(idx - r * D);
    float f1, f2, f3;
    gelu_d123(A4[idx], f1, f2, f3);
    Ab[idx] = f1 * w5[j] * ubp[r];
  }
}

// gb[q][k] = sum_j W1g[j][k] c[q][j] with W1g^T stored k-major (w1gT[k][j]).
template <int D>
__global__ __launch_bounds__(128) void boundary_adjoint_kernel(const float* __restrict__ w1gT,
                                                               const float* __restrict__ c, int n_q,
                                                               float* __restrict__ gb) {
  __shared__ float cs[D];
  const int q = blockIdx.x;
  for (int j = threadIdx.x; j < D; j += 128) cs[j] = c[(int64_t)q * D + j];
  __syncthreads();
  const int k = threadIdx.x;
  const float* w = w1gT + (int64_t)k * D;
  float s = 0.0f;
#pragma unroll 8
  for (int j = 0; j < D; ++j) s = fmaf(w[j], cs[j], s);
  gb[(int64_t)q * kNB + k] = s;
}

// ub[B_p(k)] += gb[p][k] for the placements of one sub-colour (a mod 4,
// b mod 4 fixed) among global placements q0 .. q0 + n_q - 1 of the colour
// (domains do not share memory, so only same-domain placements meet).
__global__ __launch_bounds__(128) void boundary_scatter_add_kernel(float* __restrict__ ub, AdjDomains D, int colour,
                                                                   int q0, int n_q, int sub,
                                                                   const float* __restrict__ gb) {
  const int q = blockIdx.x;
  if (q >= n_q) return;
  int lq, a, b;
  const DomEntry e = locate(D, colour, q0 + q, lq);
  placement_of(lq, colour, e.ux, a, b);
  if (((a >> 1) & 1) != (sub & 1) || ((b >> 1) & 1) != (sub >> 1)) return;
  int bi, bj;
  boundary_local(threadIdx.x, bi, bj);
  const int64_t o = e.offset + (int64_t)(kHalf * b + bj) * e.pitch + kHalf * a + bi;
  ub[o] += gb[(int64_t)q * kNB + threadIdx.x];
}

// Sum of squares of the interior of u_out into partial sums.
__global__ __launch_bounds__(256) void interior_sumsq_kernel(const float* __restrict__ u, int64_t pitch,
                                                             int nx, int ny, float* __restrict__ part) {
  __shared__ float sh[4];
  const int64_t n = (int64_t)(nx - 2) * (ny - 2);
  float acc = 0.0f;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / (nx - 2)) + 1, i = (int)(idx % (nx - 2)) + 1;
    const float v = u[(int64_t)j * pitch + i];
    acc = fmaf(v, v, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Partial sums of seed * u over every grid point (ring included).
__global__ __launch_bounds__(256) void grid_dot_kernel(const float* __restrict__ w, const float* __restrict__ u,
                                                       int64_t pitch, int nx, int ny, float* __restrict__ part) {
  __shared__ float sh[4];
  const int64_t n = (int64_t)nx * ny;
  float acc = 0.0f;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / nx), i = (int)(idx % nx);
    const int64_t o = (int64_t)j * pitch + i;
    acc = fmaf(w[o], u[o], acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void sum_parts_kernel(const float* __restrict__ part, int n, float* __restrict__ out,
                                 int accumulate) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += part[i];
    out[0] = accumulate ? out[0] + s : s;
  }
}

__global__ void fill_kernel(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// p[j * pitch + i] = v for the nx x ny grid points (row padding untouched).
__global__ void fill2d_kernel(float* __restrict__ p, int64_t pitch, int nx, int ny, float v) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx / nx, i = idx - j * nx;
    p[j * pitch + i] = v;
  }
}

static int grid_of(int64_t n, int block, int cap = 8192) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, cap));
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_of(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill2d(float* p, int64_t pitch, int ux, int uy, float v, hipStream_t s) {
  const int nx = kS * ux + 1, ny = kS * uy + 1;
  hipLaunchKernelGGL(fill2d_kernel, dim3(grid_of((int64_t)nx * ny, 256)), dim3(256), 0, s, p, pitch, nx, ny, v);
  return hipGetLastError();
}

hipError_t launch_target_coords(float* X_cross, float* X_interior, hipStream_t s) {
  hipLaunchKernelGGL(target_coords_kernel<0>, dim3(1), dim3(64), 0, s, X_cross);
  hipLaunchKernelGGL(target_coords_kernel<1>, dim3(4), dim3(256), 0, s, X_interior);
  return hipGetLastError();
}

hipError_t launch_interior_sumsq(const float* u, int64_t pitch, int ux, int uy, float* part, float* out,
                                 int accumulate, hipStream_t s) {
  const int nx = kS * ux + 1, ny = kS * uy + 1;
  const int blocks = grid_of((int64_t)(nx - 2) * (ny - 2), 256, 1024);
  hipLaunchKernelGGL(interior_sumsq_kernel, dim3(blocks), dim3(256), 0, s, u, pitch, nx, ny, part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, s, part, blocks, out, accumulate);
  return hipGetLastError();
}

hipError_t launch_grid_dot(const float* w, const float* u, int64_t pitch, int ux, int uy, float* part, float* out,
                           int accumulate, hipStream_t s) {
  const int nx = kS * ux + 1, ny = kS * uy + 1;
  const int blocks = grid_of((int64_t)nx * ny, 256, 1024);
  hipLaunchKernelGGL(grid_dot_kernel, dim3(blocks), dim3(256), 0, s, w, u, pitch, nx, ny, part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, s, part, blocks, out, accumulate);
  return hipGetLastError();
}

// Reverse one colour phase (kind ADJ_SWEEP) or one assembly colour (ADJ_SUMSQ:
// J = sum of squared interior values, u_out is the assembly; ADJ_SEED: u_out
// is the seed) for placements processed in chunks that fit the buffers in ab.
template <int D>
static hipError_t adjoint_colour_d(const NetPtrs& net, const float* whT, const AdjointBuffers& ab,
                                   const float* u_before, int64_t before_shift, const float* u_out,
                                   int64_t out_shift, float* ub, const AdjDomains& dd, int n_place, int colour,
                                   int targets, int kind, hipStream_t s) {
  const bool assembly = kind != ADJ_SWEEP;
  const int tm = assembly ? MF_INTERIOR : targets;
  const int T = tm == MF_INTERIOR ? kInterior : kCross;
  const int chunk = (int)std::max<int64_t>(1, ab.max_rows / T);
  const float* X = tm == MF_INTERIOR ? ab.X_interior : ab.X_cross;
  hipError_t e;
  for (int q0 = 0; q0 < n_place; q0 += chunk) {
    const int nq = std::min(chunk, n_place - q0);
    const int64_t n_rows = (int64_t)nq * T;
    // 1. target adjoints
    if (kind == ADJ_SUMSQ)
      hipLaunchKernelGGL((target_adjoint_kernel<1, 1>), dim3(grid_of(n_rows, 256)), dim3(256), 0, s, ub,
                         u_out, out_shift, dd, colour, q0, nq, ab.ubp);
    else if (kind == ADJ_SEED)
      hipLaunchKernelGGL((target_adjoint_kernel<1, 2>), dim3(grid_of(n_rows, 256)), dim3(256), 0, s, ub,
                         u_out, out_shift, dd, colour, q0, nq, ab.ubp);
    else if (tm == MF_CROSS)
      hipLaunchKernelGGL((target_adjoint_kernel<0, 0>), dim3(grid_of(n_rows, 256)), dim3(256), 0, s, ub,
                         u_out, out_shift, dd, colour, q0, nq, ab.ubp);
    else
      hipLaunchKernelGGL((target_adjoint_kernel<1, 0>), dim3(grid_of(n_rows, 256)), dim3(256), 0, s, ub,
                         u_out, out_shift, dd, colour, q0, nq, ab.ubp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // 2. forward of the phase from the field before it
    hipLaunchKernelGGL(gather_boundaries_kernel, dim3(grid_of((int64_t)nq * kNB, 256)), dim3(256), 0, s,
                       u_before, before_shift, dd, colour, q0, nq, ab.G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const bool gelu = ab.channels > 0;
    if (gelu) {
      if ((e = launch_embed_project(ab.params, D, ab.channels, net, ab.G, nq, nullptr, 0, 0, 0, 0, ab.C, s)) !=
          hipSuccess)
        return e;
      if ((e = launch_value_forward_gelu_saved(net, D, ab.C, X, T, nq, ab.Z, ab.Sv, s)) != hipSuccess) return e;
    } else {
      if ((e = launch_projection(net, D, ab.G, nq, ab.C, s)) != hipSuccess) return e;
      if ((e = launch_value_forward(net, D, ab.C, X, T, nq, ab.Z, s)) != hipSuccess) return e;
    }
    // 3. reverse pass to the first-layer pre-activation adjoints
    if (gelu)
      hipLaunchKernelGGL((adjoint_seed_gelu_kernel<D>), dim3(grid_of(n_rows * D, 256)), dim3(256), 0, s, ab.Sv[3],
                         net.w5, ab.ubp, n_rows, ab.Ab[0]);
    else
      hipLaunchKernelGGL((adjoint_seed_kernel<D>), dim3(grid_of(n_rows * D, 256)), dim3(256), 0, s, ab.Z[3],
                         net.w5, ab.ubp, n_rows, ab.Ab[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_value_backward(whT, D, ab.Z, gelu ? ab.Sv : nullptr, ab.Ab, n_rows, X, nq, T, ab.csum, s)) !=
        hipSuccess)
      return e;
    // 4. boundary adjoints (through the embedding for the GELU network),
    // scattered in four sub-colours
    if (gelu) {
      if ((e = launch_embed_input_adjoint(ab.params, net, D, ab.channels, ab.G, ab.csum, nq, ab.gb, s)) !=
          hipSuccess)
        return e;
    } else {
      hipLaunchKernelGGL((boundary_adjoint_kernel<D>), dim3(nq), dim3(128), 0, s, net.w1gT, ab.csum, nq, ab.gb);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int sub = 0; sub < 4; ++sub) {
      hipLaunchKernelGGL(boundary_scatter_add_kernel, dim3(nq), dim3(128), 0, s, ub, dd, colour, q0, nq, sub,
                         ab.gb);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// One colour phase (or assembly colour) reversed for every domain of the
// batch at once: doms [nd] (the caller's offsets) and qbegin [4][nd + 1] are
// device tables; u_before and u_out are read shifted by their shifts, ub is
// in the caller's frame.
hipError_t launch_adjoint_colour(const NetPtrs& net, int width, const float* whT, const AdjointBuffers& ab,
                                 const float* u_before, int64_t before_shift, const float* u_out,
                                 int64_t out_shift, float* ub, const DomEntry* doms, const int32_t* qbegin, int nd,
                                 int n_place, int colour, int targets, int kind, hipStream_t s) {
  const AdjDomains dd{doms, qbegin, nd};
  return width == 256 ? adjoint_colour_d<256>(net, whT, ab, u_before, before_shift, u_out, out_shift, ub, dd,
                                             n_place, colour, targets, kind, s)
                      : adjoint_colour_d<128>(net, whT, ab, u_before, before_shift, u_out, out_shift, ub, dd,
                                             n_place, colour, targets, kind, s);
}

}  // namespace mf

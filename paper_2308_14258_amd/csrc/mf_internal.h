// Host-side internals shared by the libmosaic translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mosaic.h"

namespace mf {

// Set the thread-local error text and return the status.
mf_status fail(mf_status s, const char* fmt, ...);

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Hidden-layer activation of the row kernels: tanh, or GELU (the
// convolutional-embedding network).
enum { ACT_TANH = 0, ACT_GELU = 1 };

// Prepared network parameters inside a workspace (offsets in bytes).
struct NetLayout {
  int width = 0, prec = 0;
  size_t w1gT = 0;   // float [128][d]: W1 boundary block, k-major
  size_t w1gb = 0;   // 16-bit W1 boundary block in MFMA operand order (MF_BF16, MF_FP16)
  size_t w1x = 0;    // float [d][2]: W1 coordinate columns
  size_t b1 = 0;     // float [d]
  size_t wh = 0;     // 3 hidden matrices, MFMA operand order (fp32, bf16 or fp16)
  size_t bh = 0;     // float [3][d]
  size_t w5 = 0;     // float [d]
  size_t b5 = 0;     // float [2]: b5, b5 + sum(w5)
  size_t end = 0;
};
NetLayout net_layout(int width, int prec, size_t base, int n_in = 128);

// Device pointers into a prepared network.
struct NetPtrs {
  const float* w1gT;
  const void* w1gb;
  const float* w1x;
  const float* b1;
  const void* wh;
  const float* bh;
  const float* w5;
  const float* b5;
};
NetPtrs net_ptrs(const NetLayout& L, const void* ws);

// Sweep workspace: prepared network, skeleton snapshot, delta partials.
struct SweepLayout {
  NetLayout net;
  size_t skel = 0;     // float [sum of n_skel over domains]
  size_t part = 0;     // float [n_domains][2][kDeltaBlocks]
  size_t dres = 0;     // float [n_domains][2]
  size_t table = 0;    // batched domains: DomEntry [n] + int32 tile prefixes [2][4][n + 1]
  size_t anext = 0;    // additive sweeps: the next field, laid out like the caller's buffer
  size_t gC = 0, gX = 0, gZ[2] = {0, 0};   // the GELU network's phase chunks (see kGeluRows)
  size_t total = 0;
};
// Rows (placement, target) per chunk of a GELU-network colour phase.
constexpr int64_t kGeluRows = 65536;
constexpr int kDeltaBlocks = 512;
int64_t skeleton_count(int ux, int uy);

// Launchers (return hipError_t of the launch).
hipError_t launch_prepare_net(const float* params, int width, int prec, const NetLayout& L,
                              void* ws, hipStream_t s);
// The hidden layers, W1x, b1, w5 and b5 of the convolutional-embedding GELU
// network (its W1 has 128 C + 2 columns and follows the convolutions), plus
// its transposed embedding block into w1gT.
hipError_t launch_prepare_net_embed(const float* params, int width, int C, const NetLayout& L, void* ws,
                                    hipStream_t s);

struct PhaseArgs {
  const float* u_in;
  float* u_out;
  int64_t pitch;
  int ux, uy, colour;
};
// One colour phase with SDNet. accumulate = assembly mode (u_out += pred / count).
hipError_t launch_phase(const NetPtrs& net, int width, int prec, int targets, bool accumulate,
                        int tile_rows, const PhaseArgs& a, hipStream_t s);

hipError_t launch_assembly_init(const float* u, float* u_out, int64_t pitch, int ux, int uy,
                                hipStream_t s);
hipError_t launch_additive_init(const float* u, float* un, int64_t pitch, int ux, int uy, int targets,
                                hipStream_t s);
hipError_t launch_additive_copy(const float* un, float* u, int64_t pitch, int ux, int uy, int targets,
                                hipStream_t s);
hipError_t launch_skeleton_snapshot(const float* u, int64_t pitch, int ux, int uy, float* skel,
                                    hipStream_t s);
hipError_t launch_delta(const float* u, int64_t pitch, int ux, int uy, const float* skel,
                        float* part, float* dres, hipStream_t s);
hipError_t launch_operator_phase(const float* Hop, int targets, bool accumulate,
                                 const PhaseArgs& a, hipStream_t s);

// One domain of a batch, as the batched colour-phase kernel reads it.
struct DomEntry {
  int64_t offset;   // first element of the domain in the packed field
  int64_t pitch;    // row pitch in floats
  int32_t ux, uy;   // units
};
SweepLayout sweep_layout(int width, int prec, const mf_domain_desc* dom, int n_domains, int mode, int embed_c = 0);
// Mixed-precision sweeps: at the targets of one colour over a batch (qbegin
// [nd + 1] placement prefixes of that colour), mode 0: corr = u - tmp, mode
// 1: u += corr; tmp and corr are indexed by the field index minus lo.
hipError_t launch_corr_targets(int targets, int mode, float* u, const float* tmp, float* corr, int64_t lo,
                               const DomEntry* doms, const int32_t* qbegin, int nd, int colour, int64_t n_place,
                               hipStream_t s);
hipError_t launch_phase_multi(const NetPtrs& net, int width, int prec, int targets, bool accumulate,
                              int tile_rows, const float* field_in, float* field_out,
                              const DomEntry* doms, const int32_t* tile_begin, int n_domains,
                              int64_t n_tiles, int colour, int n_cu, hipStream_t s);

// sdnet_forward pieces.
hipError_t launch_projection(const NetPtrs& net, int width, const float* G, int64_t n_bc,
                             float* C, hipStream_t s);
hipError_t launch_forward_rows(const NetPtrs& net, int width, int prec, const float* C,
                               const float* X, int64_t n_bc, int64_t n_pts, int x_per_bc,
                               float* U, hipStream_t s);

// Training: device buffers carved from the workspace.
// Upper bound of the fused reverse kernel's persistent grid = number of
// weight-gradient partials in the training workspace.
constexpr int kBwdGroups = 512;
// Chunks of conditions of the first-layer gradient (at most); its partials
// (kL1MaxChunks x d x (input columns + 3)) share the weight-gradient buffer.
constexpr int kL1MaxChunks = 256;
constexpr int kOutWaves = 2048;    // waves of the output-layer kernel: one partial each

struct TrainBuffers {
  float* C;          // [B][d] boundary projections (b1 included)
  float* Z[4];       // [SR][d] stream rows after layers 1..4 (z, z_x, z_y, z_L)
  float* Sv[4];      // [SR][d] saved (-, a_x, a_y, a_L) of layers 2..4 (z is Z's value row); Sv[0] null
  float* Ab[2];      // [SR][d] ping-pong pre-activation adjoints
  float* wpart;      // [kBwdGroups][d*d] weight-gradient partials
  float* bpart;      // [kBwdGroups][d]
  float* opart[2];   // [kOutWaves][d+2] output-layer partials (data, collocation)
  float* l1[2];      // [3][B][d] first-layer sums (data, collocation)
  float* grad;       // [P] gradient (used when the caller gives none)
  float* emb;        // GELU network: [B][128 C] embeddings
  float* cpart;      // GELU network: [B][10 C + 5 C^2] convolution-gradient partials
};
// Where the parameters of the network being trained sit in the flat vector.
struct TrainNet {
  const float* params;   // flat parameters (the embedding's convolutions are read from here)
  int channels;          // 0: tanh network; C: the convolutional-embedding GELU network
  int n_in;              // first-layer input columns: 128, or 128 C
  int64_t off_w1;        // W1 (d x (n_in + 2)); also the count of the convolutions' parameters
  int64_t off_w2;        // the first hidden weight matrix
  int64_t off_w5;        // the output weights
};
struct TrainLayout {
  NetLayout net;
  size_t whT = 0, C = 0, Z[4] = {0, 0, 0, 0}, Sv[4] = {0, 0, 0, 0}, Ab[2] = {0, 0};
  size_t wpart = 0, bpart = 0, opart[2] = {0, 0}, l1[2] = {0, 0}, grad = 0, emb = 0, cpart = 0, total = 0;
};
TrainLayout train_layout(const mf_sdnet_desc* desc, int64_t B, int64_t nd, int64_t nc);
TrainBuffers train_buffers(const TrainLayout& L, void* ws);

hipError_t launch_prepare_wT(const float* params, int64_t off_w2, int width, float* whT, hipStream_t s);
hipError_t launch_train_grad(const TrainNet& tn, const NetPtrs& net, int width, const float* whT,
                             const TrainBuffers& tb, const float* G, int64_t B, const float* Xd, int64_t nd,
                             int xd_per_bc, const float* Yd, const float* Xc, int64_t nc, float* grad, float* loss,
                             hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, double lr, double b1,
                       double b2, double eps, int64_t step, hipStream_t s);
// optim_kernels.hip: LAMB, one workgroup per parameter tensor. The tensor
// table travels by value (at most MF_MAX_SEGMENTS tensors); begin[n] is the
// parameter count.
struct LambSegments {
  int64_t begin[MF_MAX_SEGMENTS + 1];
  int n;
};
struct LambParams {
  // ibc1 = 1 / (1 - beta1^t), ibc2 = 1 / (1 - beta2^t): the bias corrections
  float lr, b1, omb1, b2, omb2, eps, wd, ibc1, ibc2, max_grad_norm;
  int trust;
};
hipError_t launch_lamb(float* p, float* m, float* v, const float* g, const LambSegments& S, double lr, double b1,
                       double b2, double eps, double wd, double max_grad_norm, bool trust, int64_t step,
                       hipStream_t s);
hipError_t launch_forward_derivs(const NetPtrs& net, int width, int act, const float* C, const float* X,
                                 int x_per_bc, int64_t n_bc, int64_t n_pts, float* Z0, float* Z1,
                                 float* U, float* dU, float* lapU, hipStream_t s);
hipError_t launch_value_forward_act(const NetPtrs& net, int width, int act, const float* C, const float* X,
                                    int x_per_bc, int64_t rows_per_bc, int64_t n_rows, float* const Z[4],
                                    hipStream_t s);
// embed_kernels.hip: the convolutional-embedding GELU network (activation
// MF_GELU). Its prepared network uses NetLayout with n_in = 128 C: w1gT holds
// the transposed embedding block of W1 ([128 C][d]).
constexpr int kConvK = 5;   // embedding convolutions' kernel width
int64_t embed_param_offset(int C);
hipError_t launch_prepare_w1eT(const float* params, int width, int C, float* w1eT, hipStream_t s);
hipError_t launch_embed_grad(const float* params, int width, int C, int64_t off_w1, const float* G, int64_t B,
                             const float* c0, const float* c1, float* e_out, float* part, hipStream_t s);
hipError_t launch_embed_project(const float* params, int width, int C, const NetPtrs& net, const float* G,
                                int64_t n_bc, const float* u, int64_t pitch, int ux, int colour, int q0,
                                float* Cout, hipStream_t s);
hipError_t launch_rows_output(const NetPtrs& net, int width, int targets, const float* Z, int64_t n_rows, int mode,
                              float* out, int64_t pitch, int ux, int uy, int colour, int q0, hipStream_t s);

// Adjoint of the sweep: device buffers carved from the workspace.
struct AdjointBuffers {
  float* X_cross;     // [61][2] target coordinates
  float* X_interior;  // [961][2]
  float* G;           // [max_q][128] boundary vectors of a chunk
  float* C;           // [max_q][d]
  float* ubp;         // [max_rows] target adjoints
  float* Z[4];        // [max_rows][d] activations of layers 1..4
  float* Ab[2];       // [max_rows][d] pre-activation adjoints
  float* csum;        // [3][max_q][d] first-layer sums
  float* gb;          // [max_q][128] boundary adjoints
  int64_t max_rows;
  // the GELU network (channels > 0): its parameters (for the embedding) and
  // each layer's saved pre-activations [max_rows][d]
  const float* params = nullptr;
  int channels = 0;
  float* Sv[4] = {nullptr, nullptr, nullptr, nullptr};
};
hipError_t launch_value_forward(const NetPtrs& net, int width, const float* C, const float* X, int64_t T,
                                int64_t n_bc, float* const Z[4], hipStream_t s);
hipError_t launch_value_backward(const float* whT, int width, float* const Z[4], float* const Sv[4],
                                 float* const Ab[2], int64_t n_rows, const float* X, int64_t n_bc, int64_t T,
                                 float* csum, hipStream_t s);
hipError_t launch_value_forward_gelu_saved(const NetPtrs& net, int width, const float* C, const float* X, int64_t T,
                                           int64_t n_bc, float* const Z[4], float* const Sv[4], hipStream_t s);
hipError_t launch_embed_input_adjoint(const float* params, const NetPtrs& net, int width, int C, const float* G,
                                      const float* c, int n_q, float* gb, hipStream_t s);
// io_kernels.hip: one colour's boundary gather and target scatter
hipError_t launch_gather_colour(const float* u, int64_t pitch, int ux, int colour, int64_t n_q, float* G,
                                hipStream_t s);
hipError_t launch_scatter_colour(const float* pred, int targets, float* u, int64_t pitch, int ux, int colour,
                                 int64_t n_q, hipStream_t s);
// the skeleton side layout: transposed skeleton columns (io_kernels.hip)
int64_t skel_cols_pitch(int uy);
hipError_t launch_skel_pack(const float* u, int64_t pitch, int ux, int uy, float* cols, hipStream_t s);
hipError_t launch_skel_unpack(const float* cols, float* u, int64_t pitch, int ux, int uy, hipStream_t s);
hipError_t launch_gather_skel(const float* u, int64_t pitch, const float* cols, int ux, int uy, int colour,
                              int64_t n_q, float* G, hipStream_t s);
hipError_t launch_scatter_skel(const float* pred, float* u, int64_t pitch, float* cols, int ux, int uy, int colour,
                               int64_t n_q, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill2d(float* p, int64_t pitch, int ux, int uy, float v, hipStream_t s);
hipError_t launch_target_coords(float* X_cross, float* X_interior, hipStream_t s);
hipError_t launch_interior_sumsq(const float* u, int64_t pitch, int ux, int uy, float* part, float* out,
                                 int accumulate, hipStream_t s);
hipError_t launch_grid_dot(const float* w, const float* u, int64_t pitch, int ux, int uy, float* part, float* out,
                           int accumulate, hipStream_t s);
// What an adjoint colour reverses: a sweep phase, or an assembly colour whose
// output seed is 2 u_out on the interior (ADJ_SUMSQ) or a caller's seed (ADJ_SEED).
enum { ADJ_SWEEP = 0, ADJ_SUMSQ = 1, ADJ_SEED = 2 };
hipError_t launch_adjoint_colour(const NetPtrs& net, int width, const float* whT, const AdjointBuffers& ab,
                                 const float* u_before, int64_t before_shift, const float* u_out,
                                 int64_t out_shift, float* ub, const DomEntry* doms, const int32_t* qbegin, int nd,
                                 int n_place, int colour, int targets, int kind, hipStream_t s);

}  // namespace mf

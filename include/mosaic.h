/*
 * mosaic.h -- C ABI of libmosaic: the Mosaic Flow sweep on one MI355X.
 *
 * Method: Feeney, Li, Bostanabad, Chandramowlishwaran, "Breaking Boundaries:
 * Distributed Domain Decomposition with Scalable Physics-Informed Neural PDE
 * Solvers" (SC'23, arXiv 2308.14258).
 *
 * Problem (Sec. 2.1, Eqs. 1-2): the 2-D Laplace equation with Dirichlet data
 * on a rectangle of units_x x units_y unit squares. A pretrained subdomain
 * network (SDNet, Sec. 2.4 and 3.1) maps the boundary values of a unit
 * square, sampled at 128 points, plus a point (x, y) of that square to the
 * solution there. The predictor (Sec. 4.1-4.2, Alg. 2) covers the domain
 * with overlapping unit squares placed every half unit, and sweeps: each
 * sweep runs four colour phases, and each phase gathers the boundary of every
 * same-colour placement from the global field, evaluates SDNet at that
 * placement's targets and writes the predictions back. A final assembly
 * predicts every interior point of every placement and averages the overlaps.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Field: float32, row-major, u[j * pitch + i] is the vertex (x, y) =
 *   (i / 32, j / 32) in units, 0 <= i <= 32 units_x, 0 <= j <= 32 units_y.
 *   The outer ring holds the Dirichlet data and is never written.
 * Placement (a, b), 0 <= a <= 2 units_x - 2, 0 <= b <= 2 units_y - 2, covers
 *   columns 16a .. 16a+32 and rows 16b .. 16b+32; its colour is
 *   (a mod 2) + 2 (b mod 2); a sweep runs colours 0, 1, 2, 3 in order.
 * Boundary vector (128 values): counter-clockwise from the placement's local
 *   (0, 0), 32 samples per side, each side excluding its end corner:
 *   k < 32: (k, 0); k < 64: (32, k-32); k < 96: (96-k, 32); else (0, 128-k).
 * Targets: MF_CROSS = the 61 interior points of the two centre lines (the
 *   per-iteration set of Alg. 2), MF_INTERIOR = all 31 x 31 interior points.
 *   SDNet sees local coordinates (i / 32, j / 32) in [0, 1].
 * SDNet (mf_sdnet_desc): width d in {128, 256}, depth 4 hidden layers,
 *   scalar output, in one of two architectures.
 *   MF_TANH (embed_channels = 0): tanh layers on [g, x, y]. Parameters are
 *   one flat float32 vector
 *     W1 (d x 130) | b1 (d) | W2 (d x d) | b2 | W3 | b3 | W4 | b4 | w5 (d) | b5
 *   every matrix row-major (out, in); W1 columns 0..127 act on the boundary
 *   vector, 128 on x and 129 on y.
 *   MF_GELU (embed_channels = C in 1..8): the paper's architecture (Sec. 3.1,
 *   Fig. 3): the boundary curve passes through two circular 1-D
 *   convolutions (1 -> C -> C channels, kernel 5, padding 2 wrapping around
 *   the closed curve), each followed by GELU, giving an embedding e of
 *   E = 128 C values (channel-major, e[c * 128 + k]); the layers are GELU,
 *   GELU(a) = a Phi(a) with Phi the standard normal distribution function.
 *   Parameters: Wc1 (C x 1 x 5) | bc1 (C) | Wc2 (C x C x 5) | bc2 (C) |
 *   W1 (d x (E + 2)) | b1 | W2 | b2 | W3 | b3 | W4 | b4 | w5 | b5, W1 columns
 *   0..E-1 on the embedding, E on x, E+1 on y.
 *   Either way the first layer is evaluated in the input-split form of
 *   Eq. 8: W1g g (or W1e e) + b1 once per placement (or boundary
 *   condition), plus W1x (x, y) per point. The MF_GELU network runs in
 *   MF_FP32 through mf_sweep / mf_solve (multiplicative; a placement's
 *   embedding and projection once per phase, then the value stream through
 *   MFMA GEMMs with a GELU epilogue), sdnet_forward (with its gradient
 *   and Laplacian), the training entry points (sdnet_train_step,
 *   sdnet_loss_grad; the GELU Taylor rules forward and in reverse, and the
 *   reverse through the convolutions) and mf_solve_adjoint; the autotuner,
 *   the 16-bit precisions, additive sweeps, mf_solve_mixed and
 *   mf_sweep_noalloc return MF_EUNSUPPORTED for it.
 * Precision: MF_FP32 computes every GEMM with float32 MFMA (the boundary
 *   projection on the float32 VALU). MF_BF16 rounds the GEMM operands to
 *   bf16 and accumulates in float32 on MFMA: the boundary projection
 *   W1g g (g and W1g rounded to bf16) and the three hidden d x d GEMMs
 *   (weights and the incoming activations rounded to bf16). MF_FP16 does the
 *   same with IEEE half operands (10 stored mantissa bits against bf16's 7,
 *   same MFMA rate): the gathered boundary values and every weight must lie
 *   within +-65504 (larger ones become infinite and the result is not
 *   finite; the delta test then reports MF_ENONFINITE). In all three, the
 *   field, the gather and scatter, the coordinate term W1x (x, y) + b1 of
 *   the first layer, every bias, tanh, the output layer w5 . h4 + b5 and
 *   the overlap averaging are float32. sdnet_forward computes the
 *   projection in float32 in every precision.
 *
 * Memory and streams: every pointer argument marked "device" is device
 * memory owned by the caller; "host" pointers are host memory. The library
 * never frees caller memory and allocates no device memory in any call; the
 * caller provides a workspace whose size mf_workspace_size / the *_ws_size
 * queries return (256-byte aligned). All device work is enqueued on the
 * given stream (a hipStream_t, NULL = default stream) and is asynchronous,
 * except where an entry point says it synchronises.
 *
 * Errors: every function returns mf_status. Arguments are validated on the
 * host before any device work; on failure nothing is enqueued and
 * mf_last_error() returns a thread-local description. Nothing throws or
 * aborts across this interface.
 */
#ifndef MOSAIC_H
#define MOSAIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mf_status;
enum {
  MF_OK = 0,
  MF_EINVAL = 1,         /* null/misaligned pointer, bad enum value          */
  MF_ESHAPE = 2,         /* unsupported or inconsistent sizes                */
  MF_ENOMEM = 3,         /* workspace smaller than required                  */
  MF_EDEVICE = 4,        /* no usable GPU, or a HIP call failed              */
  MF_ENONFINITE = 5,     /* delta test saw a NaN or infinity                 */
  MF_ENOTCONVERGED = 6,  /* solve hit max_sweeps with eps > 0 (opt-in flag)  */
  MF_EUNSUPPORTED = 7    /* valid request this build does not implement      */
};

enum { MF_FP32 = 0, MF_BF16 = 1, MF_FP16 = 2 };    /* precision           */
enum { MF_CROSS = 0, MF_INTERIOR = 1 };             /* target set          */
enum { MF_MULTIPLICATIVE = 0, MF_ADDITIVE = 1 };    /* sweep mode          */
enum { MF_TANH = 0, MF_GELU = 1 };                  /* activation          */
enum { MF_SOLVE_FAIL_IF_NOT_CONVERGED = 1 };        /* mf_solve flags      */
enum { MF_TILE_WIDE = 1 << 16, MF_TILE_STREAM = 1 << 17, MF_TILE_ROWSPLIT = 1 << 18,
       MF_TILE_PERSIST = 1 << 19 };                 /* tile-shape flags */

typedef struct mf_sdnet_desc {
  int32_t width;           /* d: 128 or 256                                */
  int32_t depth;           /* number of hidden layers: 4                   */
  int32_t n_boundary;      /* boundary samples: 128                        */
  int32_t activation;      /* MF_TANH or MF_GELU                           */
  int32_t embed_channels;  /* MF_TANH: 0; MF_GELU: convolution channels,
                              1..8                                         */
} mf_sdnet_desc;

typedef struct mf_domain_desc {
  int32_t units_x, units_y;  /* domain size in unit squares, each >= 1      */
  int32_t cells_per_unit;    /* 32                                          */
  int32_t stride;            /* placement stride in cells: 16               */
  int64_t pitch;             /* row pitch of the field in floats            */
  int64_t field_offset;      /* first element of this domain in the buffer  */
} mf_domain_desc;

typedef struct mf_adam {
  double lr, beta1, beta2, eps;  /* textbook Adam (Kingma and Ba); double so
                                    that 1 - beta is formed before rounding */
} mf_adam;

/* LAMB (You et al., ICLR 2020), the optimiser of the SDNet training
 * (Sec. 5.2, "Hyperparameters"). Per step t (from 1) and parameter tensor s:
 *   g <- g min(1, max_grad_norm / ||g||)   (whole gradient; max_grad_norm 0: off)
 *   m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2
 *   u <- (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps) + weight_decay w
 *   w_s <- w_s - lr r_s u_s,  r_s = ||w_s|| / ||u_s|| (1 if either is 0)
 * The trust ratio r_s is applied to every tensor when trust_without_decay
 * is 1 (LAMB as published); when it is 0, only if weight_decay != 0 (with
 * the paper's weight decay of zero the step is then Adam on the clipped
 * gradient). */
typedef struct mf_lamb {
  double lr, beta1, beta2, eps, weight_decay, max_grad_norm;
  int32_t trust_without_decay;
} mf_lamb;

/* Learning rate (Sec. 5.2): linear warm-up over W = ceil(warmup_frac x
 * total_steps) iterations to max_lr, then polynomial decay with exponent
 * `power` to end_lr at total_steps:
 *   lr(t) = max_lr t / W                                     for t <= W,
 *   lr(t) = end_lr + (max_lr - end_lr) (1 - (t - W) / (total_steps - W))^power
 *                                                            for W < t < total_steps,
 *   lr(t) = end_lr                                           from total_steps on. */
typedef struct mf_lr_schedule {
  double max_lr, warmup_frac, power, end_lr;
  int64_t total_steps;
} mf_lr_schedule;

enum { MF_MAX_SEGMENTS = 64 };                       /* tensors per LAMB step */

typedef struct mf_ctx mf_ctx;

/* Context for one device. mf_ctx_create selects `device`, checks that it is
 * a gfx950 GPU and returns MF_EDEVICE when no GPU is present. A context is
 * used by one host thread at a time. */
mf_status mf_ctx_create(int device, mf_ctx** out);
void mf_ctx_destroy(mf_ctx* ctx);
const char* mf_last_error(void);

/* mf_solve replays its sweeps (when eps = 0) from hipGraphs captured on a
 * stream owned by the context, joined to the caller's stream with events;
 * enable = 0 switches to direct launches on the caller's stream. A graph
 * holds the field and workspace addresses of the call that captured it and
 * is replayed only by later calls with the same addresses, shape, width,
 * precision and target set (at most 16 are cached per context). */
mf_status mf_ctx_graphs(mf_ctx* ctx, int32_t enable);

/* Tile shape of the colour-phase kernel for one precision: the tile height
 * (rows of (placement, target) pairs per workgroup) is 32 or 64 for MF_FP32
 * and 64, 128 or 256 for MF_BF16 and MF_FP16. Height 32 in fp32 streams the hidden
 * weights from L2; height 64 keeps each wave's slice of them in registers,
 * or streams them when or-ed with MF_TILE_STREAM (fewer registers, two
 * workgroups per CU). For MF_BF16 heights 128 and 256 may be or-ed with
 * MF_TILE_WIDE (each wave then owns 64 output columns instead of 32, halving
 * the LDS reads of the activations; not for MF_FP16), and
 * 256 | MF_TILE_ROWSPLIT selects the
 * row-split tile (each of 8 waves owns 32 rows and every unit; activations
 * stay in registers and the hidden weights stream through LDS, one
 * workgroup per CU), 128 | MF_TILE_ROWSPLIT the same tile with 4 waves (two
 * workgroups per CU; same results bit for bit); or-ed also
 * with MF_TILE_PERSIST, a batch's row-split phase runs as a persistent grid
 * (the workgroups one CU holds, per CU, walking the tiles) instead of one
 * tile per workgroup (single domains ignore the flag). 0 restores
 * the automatic choice: a tuned value from mf_autotune, else a rule on the
 * phase's rows per CU. MF_BF16 and MF_FP16: 256 | MF_TILE_ROWSPLIT from
 * 128 rows per CU up, 64 below. MF_FP32: 32 below 32 rows per CU, 64 from there, and
 * 64 | MF_TILE_STREAM for a single domain from 128 rows per CU up. */
mf_status mf_ctx_tile_rows(mf_ctx* ctx, int32_t prec, int32_t rows);

/* Autotuner: for this network, domain (or batch of n_domains domains), target
 * set and precision, time `trials` sweeps of every available tile shape with
 * hipEvents on `stream` (one warm-up sweep each, then three interleaved
 * rounds, keeping each shape's fastest round) and keep the fastest shape in
 * the context for later mf_sweep / mf_solve calls on the same configuration:
 * a single domain is matched by its units, a batch by its list of domain
 * descriptors. Candidates: MF_FP32 32, 64, 64 | MF_TILE_STREAM (batches: 32,
 * 64); MF_BF16 64, 128, 256, 128 | MF_TILE_WIDE, 256 | MF_TILE_WIDE,
 * 256 | MF_TILE_ROWSPLIT, 128 | MF_TILE_ROWSPLIT (batches also
 * 256 | MF_TILE_ROWSPLIT | MF_TILE_PERSIST); MF_FP16 the same without the MF_TILE_WIDE shapes. The sweeps run on u itself (it advances by
 * (3 trials + 1) x candidates sweeps); pass a scratch copy to keep the field.
 * rows_out (host, nullable) receives the choice. The tanh network only
 * (MF_EUNSUPPORTED for MF_GELU). Synchronises the stream. */
mf_status mf_autotune(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                      const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t prec,
                      int32_t trials, void* ws, size_t ws_bytes, void* stream, int32_t* rows_out);

/* Kernel timing, a profiling aid. While enabled, every colour-phase launch
 * of mf_sweep and mf_solve (not the assembly) is bracketed by two hipEvents
 * recorded on the stream it runs on; a replayed graph of several sweeps is
 * bracketed as a whole. mf_ctx_timing_read waits for those events and
 * returns the number of timed colour-phase launches (host, nullable), their
 * summed duration in milliseconds (host, nullable) and the SDNet point
 * evaluations they performed (host, nullable), then clears the record. */
mf_status mf_ctx_timing(mf_ctx* ctx, int32_t enable);
mf_status mf_ctx_timing_read(mf_ctx* ctx, int64_t* launches, double* total_ms, int64_t* rows);

/* Number of float32 values in the flat parameter vector (see above); -1 on
 * an invalid descriptor. Pure host function. */
int64_t mf_param_count(const mf_sdnet_desc* desc);

/* Workspace bytes needed by mf_sweep / mf_solve / mf_autotune for this
 * network, domain list (n_domains descriptors), precision, target set
 * (MF_CROSS or MF_INTERIOR) and sweep mode (MF_MULTIPLICATIVE, or
 * MF_ADDITIVE, which adds one buffer as large as the packed field for the
 * next field). A workspace sized for one set of these arguments serves any
 * call whose requirement is no larger. MF_EINVAL for unknown enum values or
 * a NULL bytes, MF_ESHAPE for an invalid domain. Pure host function. */
mf_status mf_workspace_size(const mf_sdnet_desc* desc, const mf_domain_desc* dom,
                            int32_t n_domains, int32_t prec, int32_t targets, int32_t mode,
                            size_t* bytes);

/* One colour phase (colour = 0..3) or one full sweep (colour = -1) of the
 * predictor (Sec. 4.1; the loop body of Alg. 2), updating the device field u
 * in place at the chosen targets. All placements of a phase read the field
 * as it was before the phase: same-colour placements never write a point
 * that another same-colour placement reads, so the batch equals the
 * sequential order. mode MF_ADDITIVE replaces the four ordered phases by the
 * parallel (Lions-type, Sec. 2.3) form: every placement reads the field
 * before the sweep and each target point takes the mean of the predictions
 * covering it (colour must then be -1). n_domains > 1 runs a batch of
 * independent domains packed in one buffer (dom is an array; their element
 * ranges must not overlap) with one launch per colour for the whole batch.
 * params: device, mf_param_count floats. ws: device workspace. */
mf_status mf_sweep(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params,
                   float* u, const mf_domain_desc* dom, int32_t n_domains,
                   int32_t colour, int32_t targets, int32_t mode, int32_t prec,
                   void* ws, size_t ws_bytes, void* stream);

/* mf_sweep without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation). Same arguments and result as mf_sweep in
 * MF_MULTIPLICATIVE mode (the additive mode needs a field-sized buffer and
 * is not offered here); the results are bit-identical because the same
 * kernels run. Instead of a caller's workspace it uses a static device
 * array of 1 MiB, one per GPU, held until the process ends, into which each
 * call writes the prepared network and the batch table before its kernels
 * read them. That bounds the request: the network at width 256 (about
 * 0.9 MiB in MF_FP32, 0.6 MiB in MF_BF16 or MF_FP16) plus 56 bytes per domain must
 * fit, else MF_ENOMEM with nothing enqueued (about 2,000 domains at width
 * 256 in MF_FP32). No hipMalloc, hipFree or other allocating call is made.
 * All calls on one GPU share its array, so calls that overlap in time on
 * one GPU (different streams or host threads without ordering between
 * them) race and give undefined results; calls ordered on one stream are
 * safe. Asynchronous. */
mf_status mf_sweep_noalloc(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                           const mf_domain_desc* dom, int32_t n_domains, int32_t colour, int32_t targets,
                           int32_t prec, void* stream);

/* Alg. 2 on one device: up to max_sweeps sweeps of u (in place), stopping
 * early when eps > 0 and, at a sweep whose index is a multiple of
 * check_every, the relative L2 change of the skeleton values (all grid
 * points with i or j a multiple of 16, ring included) from the previous
 * sweep drops below eps. Then, when u_out is not NULL, the final assembly
 * writes u_out (device, same layout as u): every placement predicts its 961
 * interior points from the final u and each interior point takes the mean
 * over the placements covering it; u_out's ring is copied from u.
 * sweeps_done (host, nullable) receives the number of sweeps run and
 * last_delta (host, nullable) the last delta (NaN if never evaluated).
 * Synchronises the stream when eps > 0 (one float pair read per check) and
 * when sweeps_done or last_delta is requested; otherwise asynchronous.
 * MF_ENONFINITE if a delta evaluates to NaN/inf with a nonzero reference.
 * Failure injection for tests of callers' recovery: when the environment
 * variable MF_FAULT_INJECT holds "k:c" at mf_ctx_create (k >= 1, c in 0..3),
 * a multiplicative solve on that context runs without graphs and returns
 * MF_EDEVICE just before colour phase c of sweep k, leaving u as the earlier
 * phases made it (no assembly). */
mf_status mf_solve(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params,
                   float* u, const mf_domain_desc* dom, int32_t n_domains,
                   int32_t targets, int32_t mode, int32_t prec,
                   int32_t max_sweeps, float eps, int32_t check_every, int32_t flags,
                   float* u_out, int32_t* sweeps_done, float* last_delta,
                   void* ws, size_t ws_bytes, void* stream);

/* Parses a MF_FAULT_INJECT value ("k:c", see mf_solve) into sweep k and
 * colour c (host, nullable); returns 1 when it enables injection, else 0
 * (and k = c = 0). Pure host function. */
int32_t mf_fault_inject_parse(const char* spec, int32_t* sweep, int32_t* colour);

/* Check mode: the same sweep with the subdomain solver replaced by a linear
 * operator, pred = Hop g, Hop a device float32 [T x 128] row-major matrix
 * whose rows follow the target order (CROSS: the vertical centre line
 * j = 1..31, then the horizontal line i = 1..31 without i = 16; INTERIOR:
 * row by row, i fastest). With Hop = the exact 5-point subdomain solve this
 * is classical alternating Schwarz (Sec. 2.3, Eq. 4). colour = -1 runs a
 * full sweep; colour = 4 runs the overlap-averaged assembly into u_out
 * (INTERIOR operator required). hop_rows must equal the number of targets
 * (61 or 961); it is checked because the device size of Hop is not visible
 * to the library. No workspace. */
mf_status mf_sweep_operator(mf_ctx* ctx, const float* Hop, int64_t hop_rows, int32_t targets,
                            float* u, float* u_out, const mf_domain_desc* dom, int32_t colour,
                            void* stream);

/* Placements of colour `colour` (0..3) in one domain: (units_x - (c & 1)) x
 * (units_y - (c >> 1)). Placement q of the colour is (a, b) with
 * a = (c & 1) + 2 (q mod n_a), b = (c >> 1) + 2 (q div n_a),
 * n_a = units_x - (c & 1); its 33 x 33 vertices start at grid (16 a, 16 b)
 * (Sec. 4.2). -1 on an invalid domain or colour. Pure host function. */
int64_t mf_colour_placements(const mf_domain_desc* dom, int32_t colour);

/* Local coordinates (x, y) = (i / 32, j / 32) of the target set's points in
 * the library's target order (see mf_sweep_operator), written to X_host
 * (host memory, [T][2] floats, T = 61 for MF_CROSS, 961 for MF_INTERIOR).
 * These are the X of sdnet_forward for an unfused colour phase. Pure host
 * function. */
mf_status mf_target_coords(int32_t targets, float* X_host);

/* Boundary gather of one colour phase on its own (the first step of a
 * subdomain solve in Alg. 2): G[q][k] = the field at boundary sample k of
 * placement q of the colour, k = 0..127 counter-clockwise from the
 * placement's corner (bottom edge i = 0..31, right edge j = 0..31, top edge
 * i = 32..1, left edge j = 32..1). u: device field of one domain (layout as
 * for mf_sweep; field_offset applies); G: device [mf_colour_placements][128]
 * float32, fully written (G may be NULL when the colour has no placements).
 * Asynchronous; no workspace. */
mf_status mf_gather(mf_ctx* ctx, const float* u, const mf_domain_desc* dom, int32_t colour, float* G,
                    void* stream);

/* Target scatter of one colour phase on its own (the write-back of Alg. 2):
 * the field at target t of placement q of the colour takes pred[q][t].
 * pred: device [mf_colour_placements][T] float32 in target order; u: device
 * field (only those targets are written; the placements of one colour are
 * disjoint, so every point is written at most once). With mf_gather and
 * sdnet_forward (X = mf_target_coords, shared) this is the unfused form of
 * one multiplicative colour phase of mf_sweep. pred may be NULL when the
 * colour has no placements. Asynchronous; no workspace. */
mf_status mf_scatter(mf_ctx* ctx, const float* pred, int32_t targets, float* u, const mf_domain_desc* dom,
                     int32_t colour, void* stream);

/* Skeleton side layout for the unfused colour phase. Every boundary that a
 * gather reads and every CROSS target that a scatter writes lies on the
 * skeleton: grid rows j = 16 r and grid columns i = 16 c (Sec. 4.2). The
 * rows are contiguous in the row-major field; the columns are kept
 * transposed in a caller-owned side buffer cols (device, float32,
 * mf_skeleton_cols_size floats): cols[c * cpitch + j] = u[j][16 c],
 * c = 0 .. 2 units_x, cpitch = 32 units_y + 1 rounded up to a multiple of
 * 32. Then each boundary edge and each centre line is one contiguous run.
 *   mf_skeleton_pack     fills cols from the field.
 *   mf_gather_skel       as mf_gather, reading vertical edges from cols.
 *   mf_scatter_skel      as mf_scatter with MF_CROSS targets, writing the
 *                        vertical centre line into cols, the horizontal one
 *                        into the field's row and the centre into both.
 *   mf_skeleton_unpack   writes cols back into the field's skeleton columns.
 * Between pack and unpack the skeleton state is the field's skeleton rows
 * plus cols (the field's own column entries go stale); gather -> network ->
 * scatter on this state, then unpack, gives the same field as mf_gather /
 * mf_scatter on the field, bit for bit. One domain (field_offset applies
 * to u). Asynchronous; no workspace. mf_skeleton_cols_size returns -1 on an
 * invalid domain (pure host function). */
int64_t mf_skeleton_cols_size(const mf_domain_desc* dom);
mf_status mf_skeleton_pack(mf_ctx* ctx, const float* u, const mf_domain_desc* dom, float* cols, void* stream);
mf_status mf_skeleton_unpack(mf_ctx* ctx, const float* cols, float* u, const mf_domain_desc* dom, void* stream);
mf_status mf_gather_skel(mf_ctx* ctx, const float* u, const float* cols, const mf_domain_desc* dom, int32_t colour,
                         float* G, void* stream);
mf_status mf_scatter_skel(mf_ctx* ctx, const float* pred, float* u, float* cols, const mf_domain_desc* dom,
                          int32_t colour, void* stream);

/* Workspace bytes for mf_solve_mixed. */
mf_status mf_mixed_ws_size(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int32_t n_domains,
                           int32_t targets, int32_t prec, size_t* bytes);

/* Alg. 2's sweeps in 16-bit precision (prec MF_BF16 or MF_FP16) held to the
 * float32 iteration by a correction: every refresh_every-th sweep (the
 * first included) runs each colour phase in float32 and also, from the
 * same field state, in 16 bits, and keeps the difference at every target,
 * corr_c = pred_fp32 - pred_16; the other sweeps run each phase in 16 bits
 * and add corr_c at its targets. The 16-bit map's rounding error is
 * systematic and the iteration amplifies systematic errors in its slowest
 * modes (on large domains a trained network's 16-bit fixed point lies far
 * from the float32 one); the correction, exact at each refresh and slowly
 * varying, keeps the fixed point at the float32 one. refresh_every = 1 is
 * the float32 iteration exactly (bit for bit). max_sweeps sweeps (no delta
 * test), then, when u_out is not NULL, the assembly as in mf_solve in
 * assembly_prec: MF_FP32, or prec itself (one evaluation per point, not
 * iterated, so its 16-bit rounding is not amplified: on a 64 x 64-unit
 * domain it moves the FP16 result by 4e-4 and runs 4x faster).
 * The tanh network only; single domains and batches (the correction
 * kernels take a batch's placements of a colour in one launch). The
 * workspace holds the three prepared networks (16-bit twice, float32), one
 * copy of the span the domains occupy in u and four correction fields of
 * that size. Asynchronous. */
mf_status mf_solve_mixed(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                         const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t prec,
                         int32_t max_sweeps, int32_t refresh_every, int32_t assembly_prec, float* u_out, void* ws,
                         size_t ws_bytes, void* stream);

/* Workspace bytes for mf_solve_adjoint. */
mf_status mf_adjoint_ws_size(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int32_t n_domains,
                             int32_t targets, int32_t K, int32_t ckpt_every, size_t* bytes);

/* Adjoint of Alg. 2's output with respect to its input field, float32:
 * u0_bar = (d u_out / d u0)^T uout_bar, where u_out is the overlap-averaged
 * assembly after K multiplicative sweeps of u0 (the loop and final phase of
 * Alg. 2) and uout_bar is a seed given per grid point.
 *   u0       device, read only (not modified); layout as for mf_sweep.
 *   uout_bar device seed, same layout as u0, nullable. NULL selects the
 *            objective J = sum over interior grid points of u_out^2, i.e.
 *            the seed 2 u_out on the interior and 0 on the ring. The ring of
 *            u_out is the ring of u0, so a seed's ring values are added to
 *            u0_bar's ring unchanged.
 *   u_out    device, nullable: receives the forward assembly (same layout).
 *   J        device [1], nullable: sum of squared interior values of u_out,
 *            or <uout_bar, u_out> over every grid point when a seed is
 *            given; summed over the domains of a batch.
 *   u0_bar   device, same layout as u0: fully written at the grid points
 *            (row padding untouched). Its values on the outer ring are the
 *            sensitivity to the Dirichlet data g.
 * The forward keeps field checkpoints every ckpt_every sweeps (1..1000);
 * the reverse pass runs through the assembly and every colour phase in
 * reverse order, recomputing a segment's field states from its checkpoint.
 * Each phase is reversed by reading and zeroing the target adjoints,
 * re-running the network forward from the stored field, the hand-written
 * value-stream reverse pass, gb = W1g^T sum_t ab1 (the input-split first
 * layer of Eq. 8), and a deterministic scatter-add of gb onto the placement
 * boundaries in four sub-colours. The network is evaluated in float32
 * throughout (this differentiates the MF_FP32 forward). A batch
 * (n_domains > 1) runs every domain's placements of a colour in the same
 * launches, forward and reverse. The workspace holds 2 + ceil(K / ckpt_every)
 * + 4 ckpt_every copies of the span the domains occupy in the caller's
 * buffer (from the lowest field_offset to the end of the last domain) plus
 * fixed chunk buffers (about 1.6 GB at width 256). u0, u_out, u0_bar and uout_bar
 * must be distinct buffers (MF_EINVAL). Asynchronous. */
mf_status mf_solve_adjoint(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, const float* u0,
                           const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t K,
                           int32_t ckpt_every, const float* uout_bar, float* u_out, float* J,
                           float* u0_bar, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for sdnet_forward with n_bc boundary conditions and n_pts
 * points per condition; derivatives != 0 when dU or lapU will be requested
 * (then two float32 buffers of 4 n_bc n_pts d values are included). */
mf_status sdnet_forward_ws_size(const mf_sdnet_desc* desc, int64_t n_bc, int64_t n_pts,
                                int32_t derivatives, int32_t prec, size_t* bytes);

/* N(x, g; theta) (Sec. 2.2) for n_bc boundary conditions G (device, [n_bc x
 * 128]) at points X (device): shared [n_pts x 2] when x_per_bc = 0, or per
 * condition [n_bc x n_pts x 2] when x_per_bc = 1. Writes U (device,
 * [n_bc x n_pts]). When dU (device, [n_bc x n_pts x 2], nullable) or lapU
 * (device, [n_bc x n_pts], nullable) is given, also writes the gradient and
 * the Laplacian with respect to (x, y), propagated forward through the
 * network (value, two first derivatives, Laplacian); that needs prec =
 * MF_FP32. */
mf_status sdnet_forward(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params,
                        const float* G, int64_t n_bc, const float* X, int64_t n_pts,
                        int32_t x_per_bc, float* U, float* dU, float* lapU, int32_t prec,
                        void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for sdnet_train_step / sdnet_loss_grad with B conditions,
 * nd data points and nc collocation points per condition. */
mf_status sdnet_train_ws_size(const mf_sdnet_desc* desc, int64_t B, int64_t nd, int64_t nc, size_t* bytes);

/* One physics-informed training iteration (Alg. 1 on one device, then Adam),
 * for either network (MF_TANH, or MF_GELU with its convolutional embedding):
 *   L_data = mean_{b,k} (N(Xd_{b,k}, G_b) - Yd_{b,k})^2   (data term)
 *   L_pde  = mean_{b,j} (Laplacian N(Xc_{b,j}, G_b))^2     (Eq. 3)
 * The data term is the paper's mean squared error against known solution
 * values (Sec. 5.2, "Training Methodology"); with Yd = NULL it is the
 * boundary match: the targets are G itself, so nd must be 128 and Xd holds
 * the boundary node coordinates in boundary-vector order.
 * The gradient of L_data + L_pde is accumulated from the data pass and the
 * collocation pass into one buffer; then one Adam step with bias correction
 * (step counts from 1) updates params, m and v in place (all device,
 * mf_param_count floats).
 *   G        device [B x 128] boundary vectors.
 *   Xd       device data points in the unit square: shared [nd x 2]
 *            (xd_per_bc = 0) or per condition [B x nd x 2] (xd_per_bc = 1).
 *   Yd       device [B x nd] data targets, nullable (see above).
 *   Xc       device [B x nc x 2] collocation points.
 *   loss_dev device [3]: (L_data, L_pde, L_data + L_pde) at the incoming
 *            parameters.
 *   grad_out device, nullable: when given, the gradient is written there and
 *            no update is made (m, v and hp may then be NULL).
 * Sizes: B, nd, nc >= 1 and B nd, B nc <= 2^29 (MF_ESHAPE otherwise).
 * Float32 throughout. Asynchronous. */
mf_status sdnet_train_step(mf_ctx* ctx, const mf_sdnet_desc* desc, float* params, float* m,
                           float* v, int64_t step, const mf_adam* hp, const float* G, int64_t B,
                           const float* Xd, int64_t nd, int32_t xd_per_bc, const float* Yd,
                           const float* Xc, int64_t nc, float* loss_dev, float* grad_out,
                           void* ws, size_t ws_bytes, void* stream);

/* The losses of sdnet_train_step at params and the gradient of
 * L_data + L_pde, with no parameter update: the same forward (Taylor mode)
 * and hand-written reverse pass, for callers that run their own optimiser
 * (a torch.autograd.Function, for one). Arguments as for sdnet_train_step;
 * grad_out (device, mf_param_count floats) is required and fully written;
 * loss_dev (device [3]) receives (L_data, L_pde, L_data + L_pde). Same
 * workspace size. */
mf_status sdnet_loss_grad(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, const float* G,
                          int64_t B, const float* Xd, int64_t nd, int32_t xd_per_bc, const float* Yd,
                          const float* Xc, int64_t nc, float* loss_dev, float* grad_out, void* ws,
                          size_t ws_bytes, void* stream);

/* The tensors of an SDNet's flat parameter vector, each weight matrix and
 * bias vector on its own, in layout order (the tanh network: W1, b1, W2, b2,
 * W3, b3, W4, b4, w5, b5; the GELU network: the two convolutions' kernels
 * and biases first): begin (host, capacity + 1 entries) receives the first
 * index of every tensor and, last, the parameter count; *n_segments (host)
 * the number of tensors (also when capacity is too small: MF_ESHAPE). Host
 * only. */
mf_status mf_param_segments(const mf_sdnet_desc* desc, int64_t* begin, int32_t capacity, int32_t* n_segments);

/* One LAMB step (see mf_lamb) on device vectors params, m, v (updated in
 * place) from the gradient grad (device, read only; for Alg. 1 the summed
 * data and collocation gradient of sdnet_loss_grad, averaged over devices
 * by the caller's allreduce on more than one). The tensors are given by
 * seg_begin (host, n_segments + 1 nondecreasing entries, seg_begin[0] = 0,
 * seg_begin[n_segments] = the vector length), 1 <= n_segments <=
 * MF_MAX_SEGMENTS; mf_param_segments gives an SDNet's. step counts from 1.
 * One kernel launch of n_segments workgroups on `stream`, deterministic
 * (fixed reduction order); no workspace. Asynchronous. */
mf_status sdnet_lamb_step(mf_ctx* ctx, float* params, float* m, float* v, const float* grad,
                          const int64_t* seg_begin, int32_t n_segments, int64_t step, const mf_lamb* hp,
                          void* stream);

/* The schedule's learning rate at iteration step (from 1) into *lr (host).
 * MF_EINVAL for step < 1, total_steps < 1, warmup_frac outside [0, 1],
 * max_lr or end_lr < 0, power <= 0. Host only. */
mf_status mf_lr_at(const mf_lr_schedule* sched, int64_t step, double* lr);

/* The rules for a batch batch_factor times larger (k devices, each with
 * the one-device batch; Sec. 5.2): max_lr times sqrt(batch_factor), the
 * warm-up fraction times batch_factor (at most 1); the other fields are
 * copied (the caller sets total_steps for its epochs). batch_factor > 0.
 * Host only. */
mf_status mf_lr_schedule_scaled(const mf_lr_schedule* base, double batch_factor, mf_lr_schedule* out);

#ifdef __cplusplus
}
#endif

#endif /* MOSAIC_H */

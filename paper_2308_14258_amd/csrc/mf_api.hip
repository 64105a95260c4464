// C ABI of libmosaic: argument validation, workspace layout, and the
// host-side drivers of the sweep (Alg. 2 on one device).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mf_internal.h"

namespace mf {

static thread_local char g_err[512] = "";

mf_status fail(mf_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

static mf_status ok() {
  g_err[0] = '\0';
  return MF_OK;
}

NetLayout net_layout(int width, int prec, size_t base) {
  NetLayout L;
  L.width = width;
  L.prec = prec;
  const size_t d = (size_t)width;
  size_t o = align256(base);
  L.w1gT = o; o = align256(o + 128 * d * 4);
  L.w1x = o;  o = align256(o + 2 * d * 4);
  L.b1 = o;   o = align256(o + d * 4);
  L.wh = o;   o = align256(o + 3 * d * d * (prec == MF_FP32 ? 4 : 2));
  L.bh = o;   o = align256(o + 3 * d * 4);
  L.w5 = o;   o = align256(o + d * 4);
  L.b5 = o;   o = align256(o + 4);
  L.end = o;
  return L;
}

NetPtrs net_ptrs(const NetLayout& L, const void* ws) {
  const char* b = static_cast<const char*>(ws);
  NetPtrs p;
  p.w1gT = reinterpret_cast<const float*>(b + L.w1gT);
  p.w1x = reinterpret_cast<const float*>(b + L.w1x);
  p.b1 = reinterpret_cast<const float*>(b + L.b1);
  p.wh = static_cast<const void*>(b + L.wh);
  p.bh = reinterpret_cast<const float*>(b + L.bh);
  p.w5 = reinterpret_cast<const float*>(b + L.w5);
  p.b5 = reinterpret_cast<const float*>(b + L.b5);
  return p;
}

SweepLayout sweep_layout(int width, int prec, int ux, int uy) {
  SweepLayout S;
  S.net = net_layout(width, prec, 0);
  size_t o = S.net.end;
  S.skel = o; o = align256(o + (size_t)skeleton_count(ux, uy) * 4);
  S.part = o; o = align256(o + 2 * (size_t)kDeltaBlocks * 4);
  S.dres = o; o = align256(o + 2 * 4);
  S.total = o;
  return S;
}

TrainLayout train_layout(int width, int64_t B, int64_t nc) {
  TrainLayout T;
  T.net = net_layout(width, MF_FP32, 0);
  const size_t d = (size_t)width;
  const size_t SR = (size_t)std::max<int64_t>(4 * B * nc, B * 128);   // stream rows
  const size_t chunks = (SR + 4095) / 4096;
  const size_t P = (size_t)(d * 130 + d + 3 * (d * d + d) + d + 1);
  size_t o = T.net.end;
  T.whT = o; o = align256(o + 3 * d * d * 4);
  T.C = o;   o = align256(o + (size_t)B * d * 4);
  for (int l = 0; l < 4; ++l) { T.Z[l] = o; o = align256(o + SR * d * 4); }
  for (int l = 0; l < 4; ++l) { T.Sv[l] = o; o = align256(o + SR * d * 4); }
  for (int l = 0; l < 2; ++l) { T.Ab[l] = o; o = align256(o + SR * d * 4); }
  T.wpart = o; o = align256(o + chunks * d * d * 4);
  T.bpart = o; o = align256(o + chunks * d * 4);
  for (int l = 0; l < 2; ++l) { T.opart[l] = o; o = align256(o + 2048 * (d + 2) * 4); }
  for (int l = 0; l < 2; ++l) { T.l1[l] = o; o = align256(o + 3 * (size_t)B * d * 4); }
  T.grad = o; o = align256(o + P * 4);
  T.total = o;
  return T;
}

TrainBuffers train_buffers(const TrainLayout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  TrainBuffers t;
  t.C = reinterpret_cast<float*>(b + L.C);
  for (int l = 0; l < 4; ++l) {
    t.Z[l] = reinterpret_cast<float*>(b + L.Z[l]);
    t.Sv[l] = reinterpret_cast<float*>(b + L.Sv[l]);
  }
  for (int l = 0; l < 2; ++l) {
    t.Ab[l] = reinterpret_cast<float*>(b + L.Ab[l]);
    t.opart[l] = reinterpret_cast<float*>(b + L.opart[l]);
    t.l1[l] = reinterpret_cast<float*>(b + L.l1[l]);
  }
  t.wpart = reinterpret_cast<float*>(b + L.wpart);
  t.bpart = reinterpret_cast<float*>(b + L.bpart);
  t.grad = reinterpret_cast<float*>(b + L.grad);
  return t;
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static mf_status check_desc(const mf_sdnet_desc* d) {
  if (!d) return fail(MF_EINVAL, "sdnet descriptor is NULL");
  if (d->width != 128 && d->width != 256)
    return fail(MF_ESHAPE, "sdnet width %d unsupported (128 or 256)", d->width);
  if (d->depth != 4) return fail(MF_ESHAPE, "sdnet depth %d unsupported (4)", d->depth);
  if (d->n_boundary != 128)
    return fail(MF_ESHAPE, "n_boundary %d unsupported (128)", d->n_boundary);
  if (d->activation != MF_TANH) return fail(MF_EINVAL, "activation %d unknown", d->activation);
  return MF_OK;
}

static mf_status check_prec(int prec) {
  if (prec != MF_FP32 && prec != MF_BF16) return fail(MF_EINVAL, "precision %d unknown", prec);
  return MF_OK;
}

static mf_status check_domain(const mf_domain_desc* dom, int n_domains) {
  if (!dom) return fail(MF_EINVAL, "domain descriptor is NULL");
  if (n_domains != 1)
    return fail(MF_EUNSUPPORTED, "n_domains = %d: only single-domain sweeps are implemented", n_domains);
  if (dom->units_x < 1 || dom->units_y < 1)
    return fail(MF_ESHAPE, "domain units %d x %d: each must be >= 1", dom->units_x, dom->units_y);
  if (dom->units_x > 4096 || dom->units_y > 4096)
    return fail(MF_ESHAPE, "domain units %d x %d exceed 4096", dom->units_x, dom->units_y);
  if (dom->cells_per_unit != 32) return fail(MF_ESHAPE, "cells_per_unit must be 32");
  if (dom->stride != 16) return fail(MF_ESHAPE, "placement stride must be 16 cells");
  const int64_t nx = 32LL * dom->units_x + 1, ny = 32LL * dom->units_y + 1;
  if (dom->pitch < nx) return fail(MF_ESHAPE, "pitch %lld < row length %lld", (long long)dom->pitch, (long long)nx);
  if (dom->field_offset < 0) return fail(MF_ESHAPE, "field_offset must be >= 0");
  if ((ny - 1) * dom->pitch + nx > (1LL << 40)) return fail(MF_ESHAPE, "field too large");
  return MF_OK;
}

static mf_status check_ptr(const void* p, const char* name, size_t align = 4) {
  if (!p) return fail(MF_EINVAL, "%s is NULL", name);
  if (!aligned(p, align)) return fail(MF_EINVAL, "%s is not %zu-byte aligned", name, align);
  return MF_OK;
}

static mf_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return MF_OK;
  if (!ws) return fail(MF_EINVAL, "workspace is NULL (%zu bytes needed)", need);
  if (!aligned(ws, 256)) return fail(MF_EINVAL, "workspace is not 256-byte aligned");
  if (ws_bytes < need) return fail(MF_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  return MF_OK;
}

#define MF_TRY(expr)                 \
  do {                               \
    mf_status _s = (expr);           \
    if (_s != MF_OK) return _s;      \
  } while (0)

#define MF_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) return fail(MF_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

}  // namespace mf

using namespace mf;

// A captured run of `sweeps` consecutive sweeps (4 colour-phase launches
// each) for one field / workspace / network configuration.
struct SweepGraph {
  const float* field;
  const void* ws;
  int64_t pitch;
  int ux, uy, width, prec, targets, sweeps;
  hipGraphExec_t exec;
};

struct mf_ctx {
  int device;
  int n_cu;
  hipStream_t gstream = nullptr;     // graph launches (default priority)
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<SweepGraph> graphs;
  bool use_graphs = true;
  bool timing = false;
  std::vector<hipEvent_t> events;   // pairs (start, stop) of timed launches
  std::vector<int64_t> rows;        // point evaluations of each timed record
  std::vector<int64_t> nlaunch;     // colour-phase launches in each timed record
  size_t used = 0;                  // pairs recorded since the last read
};

extern "C" {

const char* mf_last_error(void) { return g_err; }

int64_t mf_param_count(const mf_sdnet_desc* desc) {
  if (check_desc(desc) != MF_OK) return -1;
  const int64_t d = desc->width;
  return d * (desc->n_boundary + 2) + d + 3 * (d * d + d) + d + 1;
}

mf_status mf_ctx_create(int device, mf_ctx** out) {
  if (!out) return fail(MF_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0)
    return fail(MF_EDEVICE, "no GPU available (%s)", e == hipSuccess ? "0 devices" : hipGetErrorString(e));
  if (device < 0 || device >= n) return fail(MF_EDEVICE, "device %d out of range [0, %d)", device, n);
  hipDeviceProp_t prop;
  MF_HIP(hipGetDeviceProperties(&prop, device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(MF_EDEVICE, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  MF_HIP(hipSetDevice(device));
  mf_ctx* c = new (std::nothrow) mf_ctx;
  if (!c) return fail(MF_ENOMEM, "host allocation failed");
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess) {
    mf_ctx_destroy(c);
    return fail(MF_EDEVICE, "stream/event creation failed");
  }
  *out = c;
  return ok();
}

void mf_ctx_destroy(mf_ctx* ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  for (SweepGraph& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
  delete ctx;
}

mf_status mf_ctx_graphs(mf_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  ctx->use_graphs = enable != 0;
  return ok();
}

mf_status mf_ctx_timing(mf_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  ctx->timing = enable != 0;
  return ok();
}

mf_status mf_ctx_timing_read(mf_ctx* ctx, int64_t* launches, double* total_ms, int64_t* rows) {
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  double ms = 0.0;
  int64_t nrows = 0, nl = 0;
  for (size_t i = 0; i < ctx->used; ++i) {
    MF_HIP(hipEventSynchronize(ctx->events[2 * i + 1]));
    float t = 0.0f;
    MF_HIP(hipEventElapsedTime(&t, ctx->events[2 * i], ctx->events[2 * i + 1]));
    ms += t;
    nrows += ctx->rows[i];
    nl += ctx->nlaunch[i];
  }
  if (launches) *launches = nl;
  if (total_ms) *total_ms = ms;
  if (rows) *rows = nrows;
  ctx->used = 0;
  return ok();
}

mf_status mf_workspace_size(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int32_t n_domains,
                            int32_t prec, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  MF_TRY(check_domain(dom, n_domains));
  *bytes = sweep_layout(desc->width, prec, dom->units_x, dom->units_y).total;
  return ok();
}

static mf_status sweep_common_checks(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params,
                                     float* u, const mf_domain_desc* dom, int32_t n_domains,
                                     int32_t targets, int32_t mode, int32_t prec, void* ws,
                                     size_t ws_bytes, SweepLayout* L) {
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  MF_TRY(check_domain(dom, n_domains));
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(u, "u"));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (mode != MF_MULTIPLICATIVE && mode != MF_ADDITIVE) return fail(MF_EINVAL, "mode %d unknown", mode);
  if (mode == MF_ADDITIVE) return fail(MF_EUNSUPPORTED, "additive sweeps are not implemented");
  *L = sweep_layout(desc->width, prec, dom->units_x, dom->units_y);
  MF_TRY(check_ws(ws, ws_bytes, L->total));
  (void)ctx;
  return MF_OK;
}

static mf_status timing_begin(mf_ctx* ctx, hipStream_t s) {
  if (ctx->events.size() < 2 * (ctx->used + 1)) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      MF_HIP(hipEventCreate(&e));
      ctx->events.push_back(e);
    }
    ctx->rows.push_back(0);
    ctx->nlaunch.push_back(0);
  }
  MF_HIP(hipEventRecord(ctx->events[2 * ctx->used], s));
  return MF_OK;
}

static mf_status timing_end(mf_ctx* ctx, hipStream_t s, int64_t rows, int64_t launches) {
  MF_HIP(hipEventRecord(ctx->events[2 * ctx->used + 1], s));
  ctx->rows[ctx->used] = rows;
  ctx->nlaunch[ctx->used] = launches;
  ctx->used++;
  return MF_OK;
}

static int64_t phase_rows(const mf_domain_desc* dom, int colour, int targets) {
  const int64_t n_place = (int64_t)(dom->units_x - (colour & 1)) * (dom->units_y - (colour >> 1));
  return n_place * (targets == MF_INTERIOR ? 961 : 61);
}

static mf_status run_phase(mf_ctx* ctx, const NetPtrs& net, int width, int prec, int targets,
                           bool accumulate, const float* u_in, float* u_out,
                           const mf_domain_desc* dom, int colour, hipStream_t s,
                           bool allow_timing = true) {
  PhaseArgs p{u_in, u_out, dom->pitch, dom->units_x, dom->units_y, colour};
  const int64_t n_place = (int64_t)(dom->units_x - (colour & 1)) * (dom->units_y - (colour >> 1));
  const int64_t rows = n_place * ((accumulate || targets == MF_INTERIOR) ? 961 : 61);
  const int R = pick_tile_rows(width, prec, targets, rows, ctx->n_cu);
  const bool timed = allow_timing && ctx->timing && !accumulate && rows > 0;
  if (timed) MF_TRY(timing_begin(ctx, s));
  MF_HIP(launch_phase(net, width, prec, targets, accumulate, R, p, s));
  if (timed) MF_TRY(timing_end(ctx, s, rows, 1));
  return MF_OK;
}

// Cached graph of `sweeps` sweeps on ctx->gstream; captured on first use.
static mf_status sweep_graph(mf_ctx* ctx, const NetPtrs& net, const mf_sdnet_desc* desc, int prec,
                             int targets, float* field, const mf_domain_desc* dom, const void* ws,
                             int sweeps, hipGraphExec_t* out) {
  for (const SweepGraph& g : ctx->graphs) {
    if (g.field == field && g.ws == ws && g.pitch == dom->pitch && g.ux == dom->units_x &&
        g.uy == dom->units_y && g.width == desc->width && g.prec == prec && g.targets == targets &&
        g.sweeps == sweeps) {
      *out = g.exec;
      return MF_OK;
    }
  }
  if (ctx->graphs.size() >= 16) {   // bounded cache: drop the oldest entry
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  hipGraph_t graph = nullptr;
  MF_HIP(hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal));
  mf_status st = MF_OK;
  for (int k = 0; k < sweeps && st == MF_OK; ++k)
    for (int c = 0; c < 4 && st == MF_OK; ++c)
      st = run_phase(ctx, net, desc->width, prec, targets, false, field, field, dom, c, ctx->gstream,
                     false);
  hipError_t e = hipStreamEndCapture(ctx->gstream, &graph);
  if (st != MF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(MF_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MF_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
  ctx->graphs.push_back(SweepGraph{field, ws, dom->pitch, dom->units_x, dom->units_y, desc->width, prec,
                                   targets, sweeps, exec});
  *out = exec;
  return MF_OK;
}

// max_sweeps sweeps with no delta test, replayed from captured graphs of up
// to kGraphSweeps sweeps on the context's stream, ordered after and before
// the caller's stream by events.
static constexpr int kGraphSweeps = 16;
static mf_status run_sweeps_graph(mf_ctx* ctx, const NetPtrs& net, const mf_sdnet_desc* desc, int prec,
                                  int targets, float* field, const mf_domain_desc* dom, const void* ws,
                                  int max_sweeps, hipStream_t s) {
  const int full = max_sweeps / kGraphSweeps, rem = max_sweeps % kGraphSweeps;
  hipGraphExec_t g_full = nullptr, g_rem = nullptr;
  if (full > 0) MF_TRY(sweep_graph(ctx, net, desc, prec, targets, field, dom, ws, kGraphSweeps, &g_full));
  if (rem > 0) MF_TRY(sweep_graph(ctx, net, desc, prec, targets, field, dom, ws, rem, &g_rem));
  int64_t rows_sweep = 0;
  for (int c = 0; c < 4; ++c) rows_sweep += phase_rows(dom, c, targets);
  MF_HIP(hipEventRecord(ctx->fork, s));
  MF_HIP(hipStreamWaitEvent(ctx->gstream, ctx->fork, 0));
  for (int i = 0; i < full + (rem > 0 ? 1 : 0); ++i) {
    const bool last_rem = i == full;
    const int n = last_rem ? rem : kGraphSweeps;
    if (ctx->timing) MF_TRY(timing_begin(ctx, ctx->gstream));
    MF_HIP(hipGraphLaunch(last_rem ? g_rem : g_full, ctx->gstream));
    if (ctx->timing) MF_TRY(timing_end(ctx, ctx->gstream, rows_sweep * n, 4 * (int64_t)n));
  }
  MF_HIP(hipEventRecord(ctx->join, ctx->gstream));
  MF_HIP(hipStreamWaitEvent(s, ctx->join, 0));
  return MF_OK;
}

mf_status mf_sweep(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                   const mf_domain_desc* dom, int32_t n_domains, int32_t colour, int32_t targets,
                   int32_t mode, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  SweepLayout L;
  MF_TRY(sweep_common_checks(ctx, desc, params, u, dom, n_domains, targets, mode, prec, ws, ws_bytes, &L));
  if (colour < -1 || colour > 3) return fail(MF_EINVAL, "colour %d not in -1..3", colour);
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  float* field = u + dom->field_offset;
  MF_HIP(launch_prepare_net(params, desc->width, prec, L.net, ws, s));
  const NetPtrs net = net_ptrs(L.net, ws);
  for (int c = (colour < 0 ? 0 : colour); c <= (colour < 0 ? 3 : colour); ++c)
    MF_TRY(run_phase(ctx, net, desc->width, prec, targets, false, field, field, dom, c, s));
  return ok();
}

mf_status mf_solve(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                   const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t mode,
                   int32_t prec, int32_t max_sweeps, float eps, int32_t check_every, int32_t flags,
                   float* u_out, int32_t* sweeps_done, float* last_delta, void* ws, size_t ws_bytes,
                   void* stream) {
  SweepLayout L;
  MF_TRY(sweep_common_checks(ctx, desc, params, u, dom, n_domains, targets, mode, prec, ws, ws_bytes, &L));
  if (max_sweeps < 0) return fail(MF_EINVAL, "max_sweeps %d < 0", max_sweeps);
  if (!(eps >= 0.0f) || isinf(eps)) return fail(MF_EINVAL, "eps must be finite and >= 0");
  if (eps > 0.0f && check_every < 1) return fail(MF_EINVAL, "check_every %d < 1", check_every);
  if (flags & ~MF_SOLVE_FAIL_IF_NOT_CONVERGED) return fail(MF_EINVAL, "unknown flags 0x%x", flags);
  if (u_out) {
    MF_TRY(check_ptr(u_out, "u_out"));
    if (u_out == u) return fail(MF_EINVAL, "u_out must not alias u");
  }
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  float* field = u + dom->field_offset;
  MF_HIP(launch_prepare_net(params, desc->width, prec, L.net, ws, s));
  const NetPtrs net = net_ptrs(L.net, ws);
  char* wsb = static_cast<char*>(ws);
  float* skel = reinterpret_cast<float*>(wsb + L.skel);
  float* part = reinterpret_cast<float*>(wsb + L.part);
  float* dres = reinterpret_cast<float*>(wsb + L.dres);

  int done = 0;
  float last = NAN;
  bool converged = false;
  if (eps == 0.0f && ctx->use_graphs && max_sweeps > 0) {
    MF_TRY(run_sweeps_graph(ctx, net, desc, prec, targets, field, dom, ws, max_sweeps, s));
    done = max_sweeps;
  }
  for (int k = done + 1; k <= max_sweeps; ++k) {
    const bool check = eps > 0.0f && (k % check_every) == 0;
    if (check) MF_HIP(launch_skeleton_snapshot(field, dom->pitch, dom->units_x, dom->units_y, skel, s));
    for (int c = 0; c < 4; ++c)
      MF_TRY(run_phase(ctx, net, desc->width, prec, targets, false, field, field, dom, c, s));
    done = k;
    if (check) {
      MF_HIP(launch_delta(field, dom->pitch, dom->units_x, dom->units_y, skel, part, dres, s));
      float h[2];
      MF_HIP(hipMemcpyAsync(h, dres, sizeof(h), hipMemcpyDeviceToHost, s));
      MF_HIP(hipStreamSynchronize(s));
      if (h[1] == 0.0f) {
        last = INFINITY;
      } else {
        last = sqrtf(h[0]) / sqrtf(h[1]);
        if (!isfinite(last))
          return fail(MF_ENONFINITE, "delta is not finite after sweep %d", k);
      }
      if (last < eps) {
        converged = true;
        break;
      }
    }
  }
  if (u_out) {
    float* out = u_out + dom->field_offset;
    MF_HIP(launch_assembly_init(field, out, dom->pitch, dom->units_x, dom->units_y, s));
    for (int c = 0; c < 4; ++c)
      MF_TRY(run_phase(ctx, net, desc->width, prec, MF_INTERIOR, true, field, out, dom, c, s));
  }
  if (sweeps_done || last_delta) MF_HIP(hipStreamSynchronize(s));
  if (sweeps_done) *sweeps_done = done;
  if (last_delta) *last_delta = last;
  if ((flags & MF_SOLVE_FAIL_IF_NOT_CONVERGED) && eps > 0.0f && !converged)
    return fail(MF_ENOTCONVERGED, "delta %g still >= eps %g after %d sweeps", (double)last, (double)eps, done);
  return ok();
}

mf_status mf_sweep_operator(mf_ctx* ctx, const float* Hop, int64_t hop_rows, int32_t targets,
                            float* u, float* u_out, const mf_domain_desc* dom, int32_t colour,
                            void* stream) {
  MF_TRY(check_ptr(Hop, "Hop"));
  MF_TRY(check_ptr(u, "u"));
  MF_TRY(check_domain(dom, 1));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (colour < -1 || colour > 4) return fail(MF_EINVAL, "colour %d not in -1..4", colour);
  if (hop_rows != (targets == MF_CROSS ? 61 : 961))
    return fail(MF_ESHAPE, "Hop has %lld rows; the target set needs %d", (long long)hop_rows,
                targets == MF_CROSS ? 61 : 961);
  if (colour == 4) {
    if (targets != MF_INTERIOR) return fail(MF_EINVAL, "assembly needs the INTERIOR operator");
    MF_TRY(check_ptr(u_out, "u_out"));
    if (u_out == u) return fail(MF_EINVAL, "u_out must not alias u");
  }
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  float* field = u + dom->field_offset;
  if (colour == 4) {
    if (targets != MF_INTERIOR) return fail(MF_EINVAL, "assembly needs the INTERIOR operator");
    MF_TRY(check_ptr(u_out, "u_out"));
    if (u_out == u) return fail(MF_EINVAL, "u_out must not alias u");
    float* out = u_out + dom->field_offset;
    MF_HIP(launch_assembly_init(field, out, dom->pitch, dom->units_x, dom->units_y, s));
    for (int c = 0; c < 4; ++c) {
      PhaseArgs p{field, out, dom->pitch, dom->units_x, dom->units_y, c};
      MF_HIP(launch_operator_phase(Hop, MF_INTERIOR, true, p, s));
    }
    return ok();
  }
  for (int c = (colour < 0 ? 0 : colour); c <= (colour < 0 ? 3 : colour); ++c) {
    PhaseArgs p{field, field, dom->pitch, dom->units_x, dom->units_y, c};
    MF_HIP(launch_operator_phase(Hop, targets, false, p, s));
  }
  return ok();
}

// ---------------------------------------------------------------------------
// sdnet_forward
// ---------------------------------------------------------------------------
// Workspace of sdnet_forward: prepared network, projections C [n_bc][d] and,
// for derivative outputs, two stream-row buffers [4 n_bc n_pts][d].
static size_t forward_ws(int width, int prec, int64_t n_bc, int64_t n_pts, bool derivs,
                         NetLayout* Lout, size_t* c_off, size_t* z_off) {
  NetLayout L = net_layout(width, prec, 0);
  size_t o = L.end;
  *c_off = o;
  o = align256(o + (size_t)n_bc * width * 4);
  *z_off = o;
  if (derivs) o = align256(o + 2 * (size_t)4 * n_bc * n_pts * width * 4);
  if (Lout) *Lout = L;
  return o;
}

mf_status sdnet_forward_ws_size(const mf_sdnet_desc* desc, int64_t n_bc, int64_t n_pts,
                                int32_t derivatives, int32_t prec, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  if (n_bc < 0 || n_pts < 0) return fail(MF_ESHAPE, "n_bc and n_pts must be >= 0");
  size_t c_off, z_off;
  *bytes = forward_ws(desc->width, prec, n_bc, n_pts, derivatives != 0, nullptr, &c_off, &z_off);
  return ok();
}

mf_status sdnet_forward(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, const float* G,
                        int64_t n_bc, const float* X, int64_t n_pts, int32_t x_per_bc, float* U,
                        float* dU, float* lapU, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  if (n_bc < 0 || n_pts < 0) return fail(MF_ESHAPE, "n_bc and n_pts must be >= 0");
  if (x_per_bc != 0 && x_per_bc != 1) return fail(MF_EINVAL, "x_per_bc must be 0 or 1");
  if (n_bc * n_pts > (1LL << 40)) return fail(MF_ESHAPE, "too many rows");
  const bool derivs = dU || lapU;
  if (derivs && prec != MF_FP32) return fail(MF_EUNSUPPORTED, "derivative outputs need MF_FP32");
  if (n_bc == 0 || n_pts == 0) return ctx ? ok() : fail(MF_EINVAL, "ctx is NULL");
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(G, "G"));
  MF_TRY(check_ptr(X, "X"));
  MF_TRY(check_ptr(U, "U"));
  if (dU) MF_TRY(check_ptr(dU, "dU"));
  if (lapU) MF_TRY(check_ptr(lapU, "lapU"));
  NetLayout L;
  size_t c_off, z_off;
  const size_t need = forward_ws(desc->width, prec, n_bc, n_pts, derivs, &L, &c_off, &z_off);
  MF_TRY(check_ws(ws, ws_bytes, need));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_prepare_net(params, desc->width, prec, L, ws, s));
  const NetPtrs net = net_ptrs(L, ws);
  float* C = reinterpret_cast<float*>(static_cast<char*>(ws) + c_off);
  MF_HIP(launch_projection(net, desc->width, G, n_bc, C, s));
  if (!derivs) {
    MF_HIP(launch_forward_rows(net, desc->width, prec, C, X, n_bc, n_pts, x_per_bc, U, s));
  } else {
    float* Z0 = reinterpret_cast<float*>(static_cast<char*>(ws) + z_off);
    float* Z1 = Z0 + (size_t)4 * n_bc * n_pts * desc->width;
    MF_HIP(launch_forward_derivs(net, desc->width, C, X, x_per_bc, n_bc, n_pts, Z0, Z1, U, dU, lapU, s));
  }
  return ok();
}

mf_status sdnet_train_ws_size(const mf_sdnet_desc* desc, int64_t B, int64_t nc, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(check_desc(desc));
  if (B < 1 || nc < 1) return fail(MF_ESHAPE, "B and nc must be >= 1");
  if (B * nc > (1LL << 31) / 4) return fail(MF_ESHAPE, "B * nc too large");
  *bytes = train_layout(desc->width, B, nc).total;
  return ok();
}

mf_status sdnet_train_step(mf_ctx* ctx, const mf_sdnet_desc* desc, float* params, float* m, float* v,
                           int64_t step, const mf_adam* hp, const float* G, int64_t B, const float* Xb,
                           const float* Xc, int64_t nc, float* loss_dev, float* grad_out, void* ws,
                           size_t ws_bytes, void* stream) {
  MF_TRY(check_desc(desc));
  if (B < 1 || nc < 1) return fail(MF_ESHAPE, "B and nc must be >= 1");
  if (B * nc > (1LL << 31) / 4) return fail(MF_ESHAPE, "B * nc too large");
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(G, "G"));
  MF_TRY(check_ptr(Xb, "Xb"));
  MF_TRY(check_ptr(Xc, "Xc"));
  MF_TRY(check_ptr(loss_dev, "loss_dev"));
  if (grad_out) {
    MF_TRY(check_ptr(grad_out, "grad_out"));
  } else {
    MF_TRY(check_ptr(m, "m"));
    MF_TRY(check_ptr(v, "v"));
    if (!hp) return fail(MF_EINVAL, "adam hyperparameters are NULL");
    if (step < 1) return fail(MF_EINVAL, "step %lld < 1 (Adam counts from 1)", (long long)step);
    if (!(hp->lr > 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) ||
        !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) || !(hp->eps > 0.0f))
      return fail(MF_EINVAL, "adam hyperparameters out of range");
  }
  const TrainLayout L = train_layout(desc->width, B, nc);
  MF_TRY(check_ws(ws, ws_bytes, L.total));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_prepare_net(params, desc->width, MF_FP32, L.net, ws, s));
  const NetPtrs net = net_ptrs(L.net, ws);
  float* whT = reinterpret_cast<float*>(static_cast<char*>(ws) + L.whT);
  MF_HIP(launch_prepare_wT(params, desc->width, whT, s));
  const TrainBuffers tb = train_buffers(L, ws);
  float* grad = grad_out ? grad_out : tb.grad;
  MF_HIP(launch_train_grad(net, desc->width, whT, tb, G, B, Xb, Xc, nc, grad, loss_dev, s));
  if (!grad_out) {
    const double bc1 = 1.0 - pow((double)hp->beta1, (double)step);
    const double bc2 = 1.0 - pow((double)hp->beta2, (double)step);
    MF_HIP(launch_adam(params, m, v, grad, mf_param_count(desc), hp->lr, hp->beta1, hp->beta2, hp->eps,
                       (float)bc1, (float)bc2, s));
  }
  return ok();
}

}  // extern "C"
